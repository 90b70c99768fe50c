// Device bodies of the wall-normal line solves and of the refinement
// control, shared by the line-solve kernels (ibp_ytri.hip) and the
// persistent batch kernel (ibp_persist.hip).  See ibp_ytri.hip for the
// method.
#pragma once

#include "ibp_internal.hpp"

namespace ibp {

// ---------------------------------------------------------------- (0,0) mode
// Plane sums g_j of the right-hand side (FP64 row sums), the volume-weighted
// mean m = sum dyf g / (sum dyf nx nz) removed, then the face flux and the
// potential integrated upwards from the lower wall:
//   flux_0 = 0, flux_{j+1} = flux_j + dyf_j g_j,  X_0 = 0, X_j = X_{j-1} + dyc_j flux_j,
// and X shifted to zero weighted mean.  Deterministic: one wave does it with
// fixed-order sums and a Hillis-Steele scan over its 64 lane chunks, so the
// bits do not depend on the shape of the block that runs it.

// Reduction of the per-block norm partials of an x pass (fixed order for a
// given NT).
template <int NT>
__device__ __forceinline__ void reduce_parts(const ZeroArgs& Z, double* sh, double out[kPartStride]) {
  const bool ism[kPartStride] = IBP_PART_IS_MAX;
  double v[kPartStride];
#pragma unroll
  for (int q = 0; q < kPartStride; ++q) v[q] = 0.0;
  // records b, b + NT, b + 2 NT, ... in that order; four loaded at a time
  constexpr int kU = 4;
  for (long b0 = threadIdx.x; b0 < Z.nparts; b0 += kU * NT) {
    double r[kU][kPartStride];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const long b = b0 + (long)u * NT < Z.nparts ? b0 + (long)u * NT : b0;
#pragma unroll
      for (int q = 0; q < kPartStride; ++q) r[u][q] = Z.part[b * kPartStride + q];
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      if (b0 + (long)u * NT >= Z.nparts) break;
#pragma unroll
      for (int q = 0; q < kPartStride; ++q) v[q] = ism[q] ? fmax(v[q], r[u][q]) : v[q] + r[u][q];
    }
  }
  block_reduce<kPartStride, NT>(v, ism, sh);
  for (int i = 0; i < kPartStride; ++i) out[i] = v[i];
}

__device__ __forceinline__ double next_scale(double rmax) {
  if (!(rmax > 0.0) || !isfinite(rmax)) return 1.0;
  return ldexp(1.0, 20 - ilogb(rmax));
}

// Sum over the wave, lane 0's association order, broadcast to every lane.
__device__ __forceinline__ double wave_total(double v) { return __shfl(wave_sum(v), 0, kWave); }

// Exclusive prefix sum over the 64 lanes (Hillis-Steele; each lane's result
// has a fixed association order).
__device__ __forceinline__ double wave_excl_scan(double v) {
  const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    const double u = __shfl_up(v, off, kWave);
    if (lane >= off) v += u;
  }
  const double e = __shfl_up(v, 1, kWave);
  return lane > 0 ? e : 0.0;
}

// Scans of the (0,0) mode over the plane sums ghat[0..ny), run by one wave
// (so the result does not depend on the size of the block that runs it).
// Lane l owns rows [l CH, l CH + CH).  Each sweep re-reads its rows' plane
// sums (L2-resident) and recomputes the earlier sweeps' per-row values in the
// same order instead of keeping ny / 64 values per lane in registers: those
// registers would count for every block of the line-solve kernels that carry
// this path.  `p`: reduced norm partials of the right-hand side pass (used
// when Z.init).
__device__ __forceinline__ void zero_mode_scans(const ZeroArgs& Z, const double (&p)[kPartStride]) {
  const int lane = threadIdx.x & (kWave - 1), ny = Z.ny;
  const int CH = (ny + kWave - 1) / kWave;
  const int j0 = lane * CH;
  const int j1 = j0 + CH < ny ? j0 + CH : ny;
  const volatile double* gh = Z.ghat;            // written by other blocks of this launch
  double wsum = 0.0, dsum = 0.0, bad = 0.0;
  for (int j = j0; j < j1; ++j) {
    const double v = gh[j];
    wsum += Z.dyf[j] * v;
    dsum += Z.dyf[j];
    if (!isfinite(v)) bad += 1.0;
  }
  wsum = wave_total(wsum);
  dsum = wave_total(dsum);
  bad = wave_total(bad);
  const double nxnz = double(Z.nx) * double(Z.nz);
  const double m = Z.singular ? wsum / (dsum * nxnz) : 0.0;
  const double mz = m * nxnz;
  // g_j = ghat_j - m nx nz; flux at the lower face of every cell of the chunk
  double loc = 0.0;
  for (int j = j0; j < j1; ++j) loc += Z.dyf[j] * (gh[j] - mz);
  const double flux0 = wave_excl_scan(loc);
  // t_j = dyc_j flux_j (0 at the wall), summed per chunk
  double tl = 0.0;
  {
    double flux = flux0;
    for (int j = j0; j < j1; ++j) {
      const double fj = flux;
      flux += Z.dyf[j] * (gh[j] - mz);
      tl += j > 0 ? Z.dyc[j] * fj : 0.0;
    }
  }
  const double X0 = wave_excl_scan(tl);
  // X_j = running sum of t; its dyf-weighted mean
  double xw = 0.0;
  {
    double flux = flux0, X = X0;
    for (int j = j0; j < j1; ++j) {
      const double fj = flux;
      flux += Z.dyf[j] * (gh[j] - mz);
      X += j > 0 ? Z.dyc[j] * fj : 0.0;
      xw += Z.dyf[j] * X;
    }
  }
  xw = wave_total(xw);
  const double xbar = xw / dsum;
  {   // with a Dirichlet wall (0,0) goes through the line solve
    double flux = flux0, X = X0;
    for (int j = j0; j < j1; ++j) {
      const double fj = flux;
      flux += Z.dyf[j] * (gh[j] - mz);
      X += j > 0 ? Z.dyc[j] * fj : 0.0;
      const double v = Z.singular ? X - xbar : 0.0;
      Z.phi00[j] = Z.phi00_add ? Z.phi00[j] + v : v;
    }
  }
  if (Z.init && lane == 0) {
    Ctl* c = Z.ctl;
    c->done = 0;
    c->iters = 0;
    c->converged = Z.mixed ? 0 : 1;
    c->nonfinite = (bad > 0.0 || p[3] > 0.0) ? 1 : 0;
    c->scale[0] = 1.0;
    c->scale[1] = next_scale(p[2]);
    c->fnorm2 = p[1];
    c->rnorm2 = __builtin_nan("");
    c->rmax = __builtin_nan("");
    c->removed_mean = m;
    c->rel_residual = __builtin_nan("");
    c->phimean = 0.0;
    c->rel_residual_vw = __builtin_nan("");
    c->backward_error = __builtin_nan("");
    c->nhist = 0;
    c->probe = 0;
  }
}

// The (0,0) mode takes zero_blocks(ny) blocks at the start of each grid's
// line-solve launch.  Block b sums planes j = b, b + nzb, ... (one wave per
// plane: ghat[j] from the FP64 row sums in a fixed order); the block that
// finishes last (atomic ticket) then runs the scans and re-arms the ticket
// for the next launch.  A handful of blocks keeps the plane sums parallel
// while each grid pays only a handful of device-scope fences (one per
// plane, ny per launch, measured slower on batches of short grids).
// nzb: the number of blocks taking part (zero_blocks(ny) inside a line-solve
// launch; more when the (0,0) mode runs on its own).
template <int NT>
__device__ __forceinline__ void zero_mode_part(const ZeroArgs& Z, int b, int nzb) {
  __shared__ double sh[(NT / kWave) * kPartStride];
  __shared__ int last;
  constexpr int NW = NT / kWave;
  const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x) / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  for (int j = b + nzb * wave; j < Z.ny; j += nzb * NW) {
    double s = 0.0;
    const double* rs = Z.rowsum + (long)j * Z.nz;
#pragma unroll 8
    for (int k = lane; k < Z.nz; k += kWave) s += rs[k];
    s = wave_total(s);
    if (lane == 0) Z.ghat[j] = s;
  }
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) last = (atomicAdd(Z.ticket, 1) == nzb - 1);
  __syncthreads();
  if (!__builtin_amdgcn_readfirstlane(last)) return;
  __threadfence();
  double p[kPartStride];
#pragma unroll
  for (int q = 0; q < kPartStride; ++q) p[q] = 0.0;
  if (Z.init) reduce_parts<NT>(Z, sh, p);
  if (wave == 0) zero_mode_scans(Z, p);
  if (threadIdx.x == 0) atomicExch(Z.ticket, 0);
}

// ---------------------------------------------------------------- line solves
// With L = -(lambda_x + lambda_z) >= 0 and the diagonal equal to
// -(a_j + c_j + L) (the y operator is a difference of face fluxes), Thomas
// elimination is carried in eps_j = 1 + c'_j:
//   n_j = L + a_j eps_{j-1},  D_j = c_j + n_j,  eps_j = n_j / D_j,
//   d'_j = (a_j d'_{j-1} - F_j) / D_j,  X_j = d'_j + (c_j / D_j) X_{j+1},
// so every pivot D_j is a sum of non-negative terms (no cancellation, also in
// FP32).  A column's rows are split into P partitions of K rows, one per
// lane of a P-lane group inside one wave; the three recurrences are composed
// per partition (eps by 2x2 Moebius matrices with non-negative entries, d'
// and X by affine maps), chained across the
// partitions with wave shuffles (Hillis-Steele), and each lane re-sweeps its
// K rows.  The block's M columns are staged through LDS so that global loads
// and stores are M * element-size contiguous bytes per row.

// Staged tile: partition-major, then row, then column, with one pad slot
// after each partition: row r of partition pp of column m sits at slot
// pp * (K M + 1) + r M + m.  The coalesced load/store mapping (consecutive
// lanes on consecutive columns, then rows) touches consecutive slots, and
// the solve's reads (lanes on consecutive partitions of one column) are an
// odd number of slots apart, so both fall on distinct LDS banks.  P (K M + 1)
// slots: 49.7 KB at K = 12, M = 8, P = 32 in FP64, so three blocks share
// one CU's 160 KB.
template <int M, int P, int K>
__host__ __device__ constexpr long ytile_slots() { return (long)P * (K * M + 1); }

inline long ytile_slots_host(int M, int P, int K) { return (long)P * (K * M + 1); }

// Reciprocal by the hardware estimate refined with Newton's iteration
// y <- y + y (1 - x y) (two steps in FP64, one in FP32): within an ulp or
// so of 1/x for the positive, normal pivots of the line solves, at a
// fraction of the latency of a correctly rounded division.
__device__ __forceinline__ double rcp_nr(double x) {
  double y = __builtin_amdgcn_rcp(x);
  double e = fma(-x, y, 1.0);
  y = fma(y, e, y);
  e = fma(-x, y, 1.0);
  return fma(y, e, y);
}
__device__ __forceinline__ float rcp_nr(float x) {
  const float y = __builtin_amdgcn_rcpf(x);
  return fmaf(y, fmaf(-x, y, 1.0f), y);
}
// Exponent e of x = mant 2^e, 0.5 <= mant < 1, and exact scaling by 2^k.
__device__ __forceinline__ int exp2_of(double x) { return __builtin_amdgcn_frexp_exp(x); }
__device__ __forceinline__ int exp2_of(float x) { return __builtin_amdgcn_frexp_expf(x); }
__device__ __forceinline__ double scale2(double x, int k) { return __builtin_amdgcn_ldexp(x, k); }
__device__ __forceinline__ float scale2(float x, int k) { return __builtin_amdgcn_ldexpf(x, k); }

template <typename U>
__device__ __forceinline__ U shfl_up_w(U v, int d, int w) { return __shfl_up(v, d, w); }
template <typename U>
__device__ __forceinline__ U shfl_down_w(U v, int d, int w) { return __shfl_down(v, d, w); }

// Coalesced loads of the [ny][M] tile of columns q0 .. q0 + M - 1: thread
// (row0 = tid / M, lm = tid % M) loads rows row0 + P*i, i < K, all issued
// before any use (rows and columns past the end are clamped to valid
// addresses and their values discarded when staged).
template <typename T, typename U, int M, int P, int K>
__device__ __forceinline__ void ytri_load(const YArgs<T, U>& A, long q0, int lm, int row0, Cx<T> (&ld)[K]) {
  const long qc = (q0 + lm < A.Q) ? q0 + lm : A.Q - 1;
#pragma unroll
  for (int i = 0; i < K; ++i) {
    const int row = row0 + P * i;
    ld[i] = gld(gbl(A.spec) + (long)(row < A.ny ? row : A.ny - 1) * A.ps + qc);
  }
}

// The loaded values into their per-column partition slots.
template <typename T, int M, int P, int K>
__device__ __forceinline__ void ytri_stage(int ny, int lm, int row0, const Cx<T> (&ld)[K], Cx<T>* tile) {
  constexpr int PS = K * M + 1;
#pragma unroll
  for (int i = 0; i < K; ++i) {
    const int row = row0 + P * i;
    const int pp = row / K;
    tile[pp * PS + (row - pp * K) * M + lm] = row < ny ? ld[i] : Cx<T>{T(0), T(0)};
  }
}

template <typename T, typename U, int M, int P, int K, bool OUT64 = false, bool ADD = false>
__device__ __forceinline__ void ytri_solve(const YArgs<T, U>& A, long q0, Cx<T>* tile,
                                           const Cx<double> (*old)[K] = nullptr);

// Block `blk` of one grid's line-solve pass: blocks [0, zero_blocks(ny))
// run the FP64 (0,0) mode, the rest own M consecutive columns each.  With
// `kx_major` (and M dividing the row stride) the column blocks go kx group
// by kx group, all kz of one group of M kx columns before the next: the
// inverse z pass, which transforms all kz of one kx group per block and runs
// its groups in descending order, then starts on the groups written last,
// still in the Infinity Cache.  Every thread of the block calls it.
template <typename T, typename U, int M, int P, int K, bool OUT64 = false, bool ADD = false>
__device__ __forceinline__ void ytri_body(const YArgs<T, U>& A, const ZeroArgs& Z, long blk, Cx<T>* tile,
                                          bool kx_major = false) {
  constexpr int NT = M * P;
  if (A.check_done && __builtin_amdgcn_readfirstlane(A.ctl->done)) return;
  const int nzb = zero_blocks(A.ny);
  if (blk < nzb) {   // the first blocks: FP64 (0,0) mode
    zero_mode_part<NT>(Z, (int)blk, nzb);
    return;
  }
  long q0 = (blk - nzb) * M;
  const long lb = blk - nzb, nkz = A.Q / A.rs;
  if (kx_major && A.rs % M == 0) q0 = (lb % nkz) * A.rs + (lb / nkz) * M;
  if constexpr (sizeof(Cx<T>) * M == 64) {
    // Half-line column groups (64 of a row's 128 bytes): the two groups of
    // one 128-byte line go to blocks lb and lb + 8, which the round-robin
    // dispatch places on the same XCD at about the same time, so the line
    // is fetched into that XCD's L2 once.  Pairs in the block order's
    // sequence (kx-major or plain); the last nlb mod 16 blocks take the
    // remaining pairs two by two.  Rows of 128 bytes (rs a multiple of 2M)
    // give every group its sibling.
    if (A.rs % (2 * M) == 0) {
      const long nlb = A.Q / M, full = nlb / 16 * 16;
      long pair, h;
      if (lb < full) {
        pair = (lb / 16) * 8 + (lb % 8);
        h = (lb % 16) / 8;
      } else {
        pair = full / 2 + (lb - full) / 2;
        h = (lb - full) % 2;
      }
      q0 = kx_major ? (pair % nkz) * A.rs + (2 * (pair / nkz) + h) * M : (2 * pair + h) * M;
    }
  }
  const int lm = threadIdx.x % M, row0 = threadIdx.x / M;
  Cx<T> ld[K];
  ytri_load<T, U, M, P, K>(A, q0, lm, row0, ld);
  if constexpr (ADD) {
    // the FP64 values the solution is added to, loaded with the input (the
    // store loop's rows and columns)
    Cx<double> old[K];
    const long qs = q0 + lm;
    const long kz = qs / A.rs, kx = qs - kz * A.rs;
    const bool ok = qs < A.Q && kx < A.hp;
#pragma unroll
    for (int i = 0; i < K; ++i) {
      const int row = row0 + P * i;
      old[i] = (ok && row < A.ny) ? gld(gbl(A.out64) + (long)row * A.out_ps + kz * A.out_rs + kx)
                                  : Cx<double>{0.0, 0.0};
    }
    ytri_stage<T, M, P, K>(A.ny, lm, row0, ld, tile);
    __syncthreads();
    ytri_solve<T, U, M, P, K, OUT64, true>(A, q0, tile, &old);
  } else {
    ytri_stage<T, M, P, K>(A.ny, lm, row0, ld, tile);
    __syncthreads();
    ytri_solve<T, U, M, P, K, OUT64>(A, q0, tile);
  }
}

// Solve of the staged columns q0 .. q0 + M - 1 and their stores.  OUT64:
// the solution is written in FP64 to A.out64; `tile` is then the first half
// of an LDS buffer of ytile_slots FP64 entries, re-used as their FP64 staging
// once every lane has read its staged rows.
template <typename T, typename U, int M, int P, int K, bool OUT64, bool ADD>
__device__ __forceinline__ void ytri_solve(const YArgs<T, U>& A, long q0, Cx<T>* tile,
                                           const Cx<double> (*old)[K]) {
  constexpr int PS = K * M + 1;   // LDS slots per partition
  const int ny = A.ny;
  const long Q = A.Q;
  const int p = threadIdx.x % P, m = threadIdx.x / P;
  const long q = q0 + m;
  const int kz = q < Q ? (int)(q / A.rs) : 0;
  const int kx = q < Q ? (int)(q - (long)kz * A.rs) : 0;
  const bool valid = q < Q && kx < A.hp;   // row padding slots are not solved
  U L = valid ? -(gbl(A.lamx)[kx] + gbl(A.lamz)[kz]) : U(1);
  const bool zero = A.singular && q == 0;
  if (zero) L = U(1);   // singular (0,0): solved in FP64 by the (0,0)-mode blocks, zeroed here
  const int s = p * K;
  Cx<T>* my = tile + p * PS + m;   // row i of this lane's partition: my[i * M]

  // face coefficients of this lane's rows: the tables are zero-padded to
  // P*K rows, so rows past ny are decoupled (a = c = 0) and get shift 1
  U ca[K], cc[K];
#pragma unroll
  for (int i = 0; i < K; ++i) {
    ca[i] = gbl(A.ya)[s + i];
    cc[i] = gbl(A.yc)[s + i];
  }
  Cx<U> d[K];
#pragma unroll
  for (int i = 0; i < K; ++i) d[i] = Cx<U>{U(my[i * M].x), U(my[i * M].y)};
  if constexpr (OUT64) __syncthreads();   // the FP64 staging overwrites the FP32 slots
#define IBP_COEF(i, a_, c_, l_) \
  const U a_ = ca[i];           \
  const U c_ = cc[i];           \
  const U l_ = (s + (i) < ny) ? L : U(1);

  // ---- scan 1: eps_out = (mA eps_in + mB) / (mC eps_in + mD) over the
  // partition, all entries >= 0, rescaled by a power of two (exact) so that
  // mC + mD, the denominator at eps_in = 1 and positive for every row, lies
  // in [1/2, 1) (the constant term mD alone can vanish, e.g. rows with
  // shift 0 under a Neumann upper wall); a Moebius map is unchanged by a
  // common factor of its four entries
  U mA = U(1), mB = U(0), mC = U(0), mD = U(1);
#pragma unroll
  for (int i = 0; i < K; ++i) {
    IBP_COEF(i, a, c, l)
    const U n00 = a * mA + l * mC, n01 = a * mB + l * mD;
    const U n10 = a * mA + (c + l) * mC, n11 = a * mB + (c + l) * mD;
    const int ex = -exp2_of(n10 + n11);
    mA = scale2(n00, ex);
    mB = scale2(n01, ex);
    mC = scale2(n10, ex);
    mD = scale2(n11, ex);
  }
#pragma unroll
  for (int off = 1; off < P; off <<= 1) {   // inclusive prefix: mine after the earlier ones
    const U pA = shfl_up_w(mA, off, P), pB = shfl_up_w(mB, off, P);
    const U pC = shfl_up_w(mC, off, P), pD = shfl_up_w(mD, off, P);
    if (p >= off) {
      const U n00 = mA * pA + mB * pC, n01 = mA * pB + mB * pD;
      const U n10 = mC * pA + mD * pC, n11 = mC * pB + mD * pD;
      const int ex = -exp2_of(n10 + n11);
      mA = scale2(n00, ex);
      mB = scale2(n01, ex);
      mC = scale2(n10, ex);
      mD = scale2(n11, ex);
    }
  }
  {
    // eps entering the partition: the earlier composite applied to
    // eps_{-1} = 1 (the value beyond the lower wall does not depend on X_0)
    const U eA = shfl_up_w(mA, 1, P), eB = shfl_up_w(mB, 1, P);
    const U eC = shfl_up_w(mC, 1, P), eD = shfl_up_w(mD, 1, P);
    U e = (eA + eB) / (eC + eD);
    if (p == 0) e = U(1);
    // with the pivots known, keep a_j / D_j, c_j / D_j and F_j / D_j only
    // (both later recurrences use nothing else)
#pragma unroll
    for (int i = 0; i < K; ++i) {
      IBP_COEF(i, a, c, l)
      const U n = l + a * e;
      const U r = rcp_nr(c + n);
      e = n * r;
      ca[i] = a * r;
      cc[i] = c * r;
      d[i] = cscale(d[i], r);
    }
  }
  // ---- scan 2: d'_out = mu d'_in + nu over the partition
  {
    U mu = U(1);
    Cx<U> nu{U(0), U(0)};
#pragma unroll
    for (int i = 0; i < K; ++i) {
      const U mi = ca[i];
      mu = mi * mu;
      nu = csub(cscale(nu, mi), d[i]);
    }
#pragma unroll
    for (int off = 1; off < P; off <<= 1) {
      const U pm = shfl_up_w(mu, off, P);
      const U px = shfl_up_w(nu.x, off, P), py = shfl_up_w(nu.y, off, P);
      if (p >= off) {
        nu = Cx<U>{mu * px + nu.x, mu * py + nu.y};
        mu = mu * pm;
      }
    }
    Cx<U> prev{shfl_up_w(nu.x, 1, P), shfl_up_w(nu.y, 1, P)};
    if (p == 0) prev = Cx<U>{U(0), U(0)};
#pragma unroll
    for (int i = 0; i < K; ++i) {
      d[i] = csub(cscale(prev, ca[i]), d[i]);
      prev = d[i];
    }
  }
  // ---- scan 3 (upwards): X_first = T X_below + S over the partition
  {
    U Tt = U(1);
    Cx<U> S{U(0), U(0)};
#pragma unroll
    for (int i = K - 1; i >= 0; --i) {
      const U tau = cc[i];
      Tt = tau * Tt;
      S = cadd(d[i], cscale(S, tau));
    }
#pragma unroll
    for (int off = 1; off < P; off <<= 1) {   // inclusive suffix: mine before the later ones
      const U nT = shfl_down_w(Tt, off, P);
      const U sx = shfl_down_w(S.x, off, P), sy = shfl_down_w(S.y, off, P);
      if (p + off < P) {
        S = Cx<U>{Tt * sx + S.x, Tt * sy + S.y};
        Tt = Tt * nT;
      }
    }
    Cx<U> nxt{shfl_down_w(S.x, 1, P), shfl_down_w(S.y, 1, P)};
    if (p == P - 1) nxt = Cx<U>{U(0), U(0)};
#pragma unroll
    for (int i = K - 1; i >= 0; --i) {
      d[i] = cadd(d[i], cscale(nxt, cc[i]));
      nxt = d[i];
    }
  }
#undef IBP_COEF
  if constexpr (OUT64) {
    Cx<double>* t64 = reinterpret_cast<Cx<double>*>(tile);
    Cx<double>* my64 = t64 + p * PS + m;
#pragma unroll
    for (int i = 0; i < K; ++i) my64[i * M] = zero ? Cx<double>{0.0, 0.0} : Cx<double>{double(d[i].x), double(d[i].y)};
    __syncthreads();
    const int mm = threadIdx.x % M, row0 = threadIdx.x / M;
    const long qs = q0 + mm;
    const long kz = qs / A.rs, kx = qs - kz * A.rs;
    if (qs < Q && kx < A.hp) {
      const double inv_s = ADD ? 1.0 / A.ctl->scale[A.add_iter & 1] : 1.0;
#pragma unroll
      for (int i = 0; i < K; ++i) {
        const int row = row0 + P * i;
        const int pp = row / K;
        Cx<double> v = t64[pp * PS + (row - pp * K) * M + mm];
        if constexpr (ADD) v = cadd((*old)[i], cscale(v, inv_s));
        if (row < ny) gst(gbl(A.out64) + (long)row * A.out_ps + kz * A.out_rs + kx, v);
      }
    }
    return;
  }
#pragma unroll
  for (int i = 0; i < K; ++i) my[i * M] = zero ? Cx<T>{T(0), T(0)} : Cx<T>{T(d[i].x), T(d[i].y)};
  __syncthreads();
  {
    const int mm = threadIdx.x % M, row0 = threadIdx.x / M;
    const long qs = q0 + mm;
    if (qs < Q && qs % A.rs < A.hp) {
#pragma unroll
      for (int i = 0; i < K; ++i) {
        const int row = row0 + P * i;
        const int pp = row / K;
        const Cx<T> v = tile[pp * PS + (row - pp * K) * M + mm];
        if (row < ny) gst(gbl(A.spec) + (long)row * A.ps + qs, v);
      }
    }
  }
}

// ---------------------------------------------------------------- control
// Convergence test of a refinement pass (one block): reduce the partials of
// the residual pass, record ||r||/||f - m||, and either stop the refinement or
// set the FP32 input scale of the next pass.
template <int NT>
__device__ __forceinline__ void check_body(const ZeroArgs& Z, double* sh) {
  if (__builtin_amdgcn_readfirstlane(Z.ctl->done)) return;
  if (Z.probe && !__builtin_amdgcn_readfirstlane(Z.ctl->probe)) return;
  double p[kPartStride];
  reduce_parts<NT>(Z, sh, p);
  if (threadIdx.x != 0) return;
  Ctl* c = Z.ctl;
  auto ratio = [](double num2, double den2) {
    if (den2 > 0.0) return sqrt(num2 / den2);
    return num2 == 0.0 ? 0.0 : __builtin_inf();
  };
  const double rel = ratio(p[0], p[1]);
  // normwise backward error: ||r||_inf / (||L_h||_inf ||phi||_inf + ||f - m||_inf)
  const double den = Z.lnorm * p[7] + p[8];
  const double eta = den > 0.0 ? p[2] / den : (p[2] == 0.0 ? 0.0 : __builtin_inf());
  c->rnorm2 = p[0];
  c->fnorm2 = p[1];
  c->rmax = p[2];
  c->rel_residual = rel;
  c->rel_residual_vw = ratio(p[5], p[6]);
  c->backward_error = eta;
  // the residual of the iterate after iter - 1 corrections
  if (Z.iter - 1 < kHistMax) c->hist[Z.iter - 1] = rel;
  c->nhist = Z.iter < kHistMax ? Z.iter : kHistMax;
  // the mean of a Neumann-Neumann iterate is fixed to zero; with a
  // Dirichlet wall the solution's mean is part of it
  c->phimean = Z.singular ? p[4] / (Z.dyf_sum * double(Z.nx) * double(Z.nz)) : 0.0;
  if (p[3] > 0.0) c->nonfinite = 1;
  if (rel <= Z.rtol && !Z.nostop) {
    c->done = 1;
    c->converged = 1;
  } else if (eta <= kEtaFloor && !Z.nostop) {   // at the FP64 floor: corrections cannot lower the residual
    c->done = 1;
    c->converged = 2;
  } else if (Z.probe) {
    // not converged: the full residual pass of the same iterate follows and
    // its check decides the next step
  } else if (!Z.nostop && (Z.final_pass || !(rel > Z.rtol))) {   // last pass, or a NaN residual
    c->done = 1;
    c->converged = 0;
  } else {
    c->iters = Z.iter;
    c->scale[(Z.iter + 1) & 1] = next_scale(p[2]);
    // Predict the residual after this correction from the contraction so
    // far (the first correction: the initial solve's own relative
    // residual); when it should meet rtol, the next pass tests the
    // corrected iterate with a residual-only pass first and skips the
    // residual transform if it has converged.
    const double prev = Z.iter >= 2 && Z.iter - 2 < kHistMax ? c->hist[Z.iter - 2] : 1.0;
    const double pred = rel * (rel / prev);
    c->probe = pred <= Z.rtol ? 1 : 0;
  }
}

}  // namespace ibp

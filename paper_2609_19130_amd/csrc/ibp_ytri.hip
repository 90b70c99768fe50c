// Wall-normal line solves, one tridiagonal system per horizontal Fourier mode
// (paper: after the FFTs, independent tridiagonal systems remain along x3 for
// each horizontal mode; "Fluid domain" parallelisation subsection), plus the
// singular (0,0) mode in FP64 and the refinement control.
//
// Mode (kx, kz) solves  a_j X_{j-1} + (b_j + lx(kx) + lz(kz)) X_j + c_j X_{j+1} = F_j,
// j = 0..ny-1, real coefficients, complex right-hand side, a_0 = c_{ny-1} = 0
// (homogeneous Neumann walls).
//
// Block decomposition: a block owns M consecutive spectral columns; the
// P = 256/M threads of one column each own K consecutive rows (rows past ny
// are decoupled padding).  All K rows are loaded before any arithmetic, so
// every thread keeps K loads in flight, and consecutive threads read
// consecutive columns (16*M-byte segments in FP64).
#include "ibp_internal.hpp"

namespace ibp {

// ---------------------------------------------------------------- (0,0) mode
// Plane sums g_j of the right-hand side (FP64 row sums), the volume-weighted
// mean m = sum dyf g / (sum dyf nx nz) removed, then the face flux and the
// potential integrated upwards from the lower wall:
//   flux_0 = 0, flux_{j+1} = flux_j + dyf_j g_j,  X_0 = 0, X_j = X_{j-1} + dyc_j flux_j,
// and X shifted to zero weighted mean.  Deterministic: fixed-order sums and
// a Hillis-Steele scan over the 256 thread chunks.
__device__ double block_excl_scan(double v, double* sc) {
  const int t = threadIdx.x;
  sc[t] = v;
  __syncthreads();
  for (int off = 1; off < kThreads; off <<= 1) {
    const double add = t >= off ? sc[t - off] : 0.0;
    __syncthreads();
    sc[t] += add;
    __syncthreads();
  }
  const double r = t > 0 ? sc[t - 1] : 0.0;
  __syncthreads();
  return r;
}

__device__ double block_sum_det(double v, double* sh) {
  bool ism[1] = {false};
  double a[1] = {v};
  block_reduce<1>(a, ism, sh);
  return a[0];
}

__device__ void reduce_parts(const ZeroArgs& Z, double* sh, double out[4]) {
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  for (long b = threadIdx.x; b < Z.nparts; b += kThreads) {
    const double* p = Z.part + b * kPartStride;
    v[0] += p[0];
    v[1] += p[1];
    v[2] = fmax(v[2], p[2]);
    v[3] += p[3];
  }
  const bool ism[4] = {false, false, true, false};
  block_reduce<4>(v, ism, sh);
  for (int i = 0; i < 4; ++i) out[i] = v[i];
}

__device__ double next_scale(double rmax) {
  if (!(rmax > 0.0) || !isfinite(rmax)) return 1.0;
  return ldexp(1.0, 20 - ilogb(rmax));
}

__device__ void zero_mode_block(const ZeroArgs& Z) {
  __shared__ double sc[kThreads];
  __shared__ double sh[16];
  const int t = threadIdx.x, ny = Z.ny, nz = Z.nz;
  const int CH = (ny + kThreads - 1) / kThreads;
  const int j0 = t * CH;
  double g[kMaxYChunk];
  double wsum = 0.0, dsum = 0.0, bad = 0.0;
#pragma unroll
  for (int c = 0; c < kMaxYChunk; ++c) {
    g[c] = 0.0;
    const int j = j0 + c;
    if (c < CH && j < ny) {
      double s = 0.0;
      const double* rs = Z.rowsum + (long)j * nz;
      for (int k = 0; k < nz; ++k) s += rs[k];
      g[c] = s;
      wsum += Z.dyf[j] * s;
      dsum += Z.dyf[j];
      if (!isfinite(s)) bad += 1.0;
    }
  }
  wsum = block_sum_det(wsum, sh);
  dsum = block_sum_det(dsum, sh);
  bad = block_sum_det(bad, sh);
  const double nxnz = double(Z.nx) * double(Z.nz);
  const double m = wsum / (dsum * nxnz);
  // flux at the lower face of every cell of the chunk
  double loc = 0.0;
#pragma unroll
  for (int c = 0; c < kMaxYChunk; ++c) {
    const int j = j0 + c;
    if (c < CH && j < ny) {
      g[c] -= m * nxnz;
      loc += Z.dyf[j] * g[c];
    }
  }
  double flux = block_excl_scan(loc, sc);
  double tl = 0.0;
#pragma unroll
  for (int c = 0; c < kMaxYChunk; ++c) {      // g[c] <- dyc_j flux_j
    const int j = j0 + c;
    if (c < CH && j < ny) {
      const double fj = flux;
      flux += Z.dyf[j] * g[c];
      g[c] = j > 0 ? Z.dyc[j] * fj : 0.0;
      tl += g[c];
    }
  }
  double X = block_excl_scan(tl, sc);
  double xw = 0.0;
#pragma unroll
  for (int c = 0; c < kMaxYChunk; ++c) {      // g[c] <- X_j
    const int j = j0 + c;
    if (c < CH && j < ny) {
      X += g[c];
      g[c] = X;
      xw += Z.dyf[j] * X;
    }
  }
  xw = block_sum_det(xw, sh);
  const double xbar = xw / dsum;
#pragma unroll
  for (int c = 0; c < kMaxYChunk; ++c) {
    const int j = j0 + c;
    if (c < CH && j < ny) Z.phi00[j] = g[c] - xbar;
  }
  if (Z.init) {
    double p[4];
    reduce_parts(Z, sh, p);
    if (t == 0) {
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
    }
  }
}

// ---------------------------------------------------------------- line solves
// With L = -(lambda_x + lambda_z) >= 0 and the diagonal equal to
// -(a_j + c_j + L) (the y operator is a difference of face fluxes), Thomas
// elimination is carried in eps_j = 1 + c'_j:
//   n_j = L + a_j eps_{j-1},  D_j = c_j + n_j,  eps_j = n_j / D_j,
//   d'_j = (a_j d'_{j-1} - F_j) / D_j,  X_j = d'_j + (c_j / D_j) X_{j+1},
// so every pivot D_j is a sum of non-negative terms (no cancellation, also in
// FP32).  Across the P row blocks of a column the three recurrences are
// composed: eps by 2x2 Moebius matrices with non-negative entries, d' and X
// by affine maps with coefficients in [0, 1]; one thread per column chains
// the P block composites in LDS, then every thread re-sweeps its K rows.
template <typename T, typename U, int K, int M>
__global__ __launch_bounds__(kThreads) void k_ytri(YArgs<T, U> A, ZeroArgs Z) {
  constexpr int P = kThreads / M;
  __shared__ U sA[M][P + 1], sB[M][P + 1], sC[M][P + 1];
  __shared__ Cx<U> sD[M][P + 1];
  if (blockIdx.x == gridDim.x - 1) {
    if (!(A.check_done && A.ctl->done)) zero_mode_block(Z);
    return;
  }
  if (A.check_done && A.ctl->done) return;
  const int m = threadIdx.x % M, p = threadIdx.x / M;
  const long q = (long)blockIdx.x * M + m;
  const bool valid = q < A.Q;
  const int kz = valid ? (int)(q / A.hp) : 0;
  const int kx = valid ? (int)(q - (long)kz * A.hp) : 0;
  U L = valid ? -(A.lamx[kx] + A.lamz[kz]) : U(1);
  if (q == 0) L = U(1);   // (0,0) is singular: solved in FP64 by the last block, zeroed here
  const int s = p * K, ny = A.ny;
  const long Q = A.Q;
  const U* __restrict__ ya = A.ya;
  const U* __restrict__ yc = A.yc;

  Cx<U> d[K];
#pragma unroll
  for (int i = 0; i < K; ++i) {
    const int row = s + i;
    Cx<T> v{T(0), T(0)};
    if (valid && row < ny) v = A.spec[(long)row * Q + q];
    d[i] = Cx<U>{U(v.x), U(v.y)};
  }
  // rows past ny are decoupled padding: a = c = 0, shift 1
#define IBP_COEF(i, a_, c_, l_)           \
  const bool in_ = (s + (i)) < ny;        \
  const U a_ = in_ ? ya[s + (i)] : U(0);  \
  const U c_ = in_ ? yc[s + (i)] : U(0);  \
  const U l_ = in_ ? L : U(1);

  // ---- scan 1: eps_out = (mA eps_in + mB) / (mC eps_in + 1) over the block
  U mA = U(1), mB = U(0), mC = U(0);
#pragma unroll
  for (int i = 0; i < K; ++i) {
    IBP_COEF(i, a, c, l)
    const U n00 = a * mA + l * mC, n01 = a * mB + l;
    const U n10 = a * mA + (c + l) * mC, n11 = a * mB + (c + l);
    const U inv = U(1) / n11;
    mA = n00 * inv;
    mB = n01 * inv;
    mC = n10 * inv;
  }
  sA[m][p] = mA;
  sB[m][p] = mB;
  sC[m][p] = mC;
  __syncthreads();
  if (p == 0) {
    U e = U(0);
    for (int pp = 0; pp < P; ++pp) {
      const U a_ = sA[m][pp], b_ = sB[m][pp], c_ = sC[m][pp];
      sA[m][pp] = e;
      e = (a_ * e + b_) / (c_ * e + U(1));
    }
  }
  __syncthreads();
  U rD[K];
  {
    U e = sA[m][p];
#pragma unroll
    for (int i = 0; i < K; ++i) {
      IBP_COEF(i, a, c, l)
      const U n = l + a * e;
      rD[i] = U(1) / (c + n);
      e = n * rD[i];
    }
  }
  __syncthreads();
  // ---- scan 2: d'_out = mu d'_in + nu over the block
  {
    U mu = U(1);
    Cx<U> nu{U(0), U(0)};
#pragma unroll
    for (int i = 0; i < K; ++i) {
      IBP_COEF(i, a, c, l)
      (void)c;
      (void)l;
      const U mi = a * rD[i];
      mu = mi * mu;
      nu = csub(cscale(nu, mi), cscale(d[i], rD[i]));
    }
    sA[m][p] = mu;
    sD[m][p] = nu;
  }
  __syncthreads();
  if (p == 0) {
    Cx<U> x{U(0), U(0)};
    for (int pp = 0; pp < P; ++pp) {
      const U mu_ = sA[m][pp];
      const Cx<U> nu_ = sD[m][pp];
      sD[m][pp] = x;
      x = cadd(cscale(x, mu_), nu_);
    }
  }
  __syncthreads();
  {
    Cx<U> prev = sD[m][p];
#pragma unroll
    for (int i = 0; i < K; ++i) {
      IBP_COEF(i, a, c, l)
      (void)c;
      (void)l;
      d[i] = cscale(csub(cscale(prev, a), d[i]), rD[i]);
      prev = d[i];
    }
  }
  __syncthreads();
  // ---- scan 3 (upwards): X_first = T X_below + S over the block
  {
    U Tt = U(1);
    Cx<U> S{U(0), U(0)};
#pragma unroll
    for (int i = K - 1; i >= 0; --i) {
      IBP_COEF(i, a, c, l)
      (void)a;
      (void)l;
      const U tau = c * rD[i];
      Tt = tau * Tt;
      S = cadd(d[i], cscale(S, tau));
    }
    sA[m][p] = Tt;
    sD[m][p] = S;
  }
  __syncthreads();
  if (p == 0) {
    Cx<U> x{U(0), U(0)};
    for (int pp = P - 1; pp >= 0; --pp) {
      const U T_ = sA[m][pp];
      const Cx<U> S_ = sD[m][pp];
      sD[m][pp] = x;
      x = cadd(cscale(x, T_), S_);
    }
  }
  __syncthreads();
  if (!valid) return;
  {
    Cx<U> nxt = sD[m][p];
#pragma unroll
    for (int i = K - 1; i >= 0; --i) {
      IBP_COEF(i, a, c, l)
      (void)a;
      (void)l;
      d[i] = cadd(d[i], cscale(nxt, c * rD[i]));
      nxt = d[i];
    }
  }
#undef IBP_COEF
  const bool zero = (q == 0);
#pragma unroll
  for (int i = 0; i < K; ++i) {
    const int row = s + i;
    if (row < ny) {
      const Cx<U> x = zero ? Cx<U>{U(0), U(0)} : d[i];
      A.spec[(long)row * Q + q] = Cx<T>{T(x.x), T(x.y)};
    }
  }
}

// ---------------------------------------------------------------- control
// Convergence test of a refinement pass (one block): reduce the partials of
// the residual pass, record ||r||/||f - m||, and either stop the refinement or
// set the FP32 input scale of the next pass.
__global__ __launch_bounds__(kThreads) void k_check(ZeroArgs Z) {
  __shared__ double sh[16];
  if (Z.ctl->done) return;
  double p[4];
  reduce_parts(Z, sh, p);
  if (threadIdx.x != 0) return;
  Ctl* c = Z.ctl;
  double rel;
  if (p[1] > 0.0)
    rel = sqrt(p[0] / p[1]);
  else
    rel = (p[0] == 0.0) ? 0.0 : __builtin_inf();
  c->rnorm2 = p[0];
  c->fnorm2 = p[1];
  c->rmax = p[2];
  c->rel_residual = rel;
  if (p[3] > 0.0) c->nonfinite = 1;
  if (Z.final_pass || !(rel > Z.rtol)) {
    c->done = 1;
    c->converged = (rel <= Z.rtol) ? 1 : 0;
  } else {
    c->iters = Z.iter;
    c->scale[(Z.iter + 1) & 1] = next_scale(p[2]);
  }
}

hipError_t launch_check(const ZeroArgs& z, hipStream_t s) {
  hipLaunchKernelGGL(k_check, dim3(1), dim3(kThreads), 0, s, z);
  return hipGetLastError();
}

// ---------------------------------------------------------------- dispatch
static constexpr int kKs[] = {2, 4, 6, 8, 12, 16, 24};

bool ytri_shape(int ny, int* M, int* K) {
  if (ny < 2 || ny > kMaxNy) return false;
  int m = 16;
  while (m > 1 && (kThreads / m) * 24 < ny) m /= 2;
  const int P = kThreads / m;
  const int need = (ny + P - 1) / P;
  for (int k : kKs) {
    if (k >= need) {
      *M = m;
      *K = k;
      return true;
    }
  }
  return false;
}

template <typename T, typename U, int M>
static hipError_t launch_ytri_m(int K, const YArgs<T, U>& a, const ZeroArgs& z, hipStream_t s, dim3 grid) {
  dim3 block(kThreads);
  switch (K) {
    case 2: hipLaunchKernelGGL((k_ytri<T, U, 2, M>), grid, block, 0, s, a, z); break;
    case 4: hipLaunchKernelGGL((k_ytri<T, U, 4, M>), grid, block, 0, s, a, z); break;
    case 6: hipLaunchKernelGGL((k_ytri<T, U, 6, M>), grid, block, 0, s, a, z); break;
    case 8: hipLaunchKernelGGL((k_ytri<T, U, 8, M>), grid, block, 0, s, a, z); break;
    case 12: hipLaunchKernelGGL((k_ytri<T, U, 12, M>), grid, block, 0, s, a, z); break;
    case 16: hipLaunchKernelGGL((k_ytri<T, U, 16, M>), grid, block, 0, s, a, z); break;
    case 24: hipLaunchKernelGGL((k_ytri<T, U, 24, M>), grid, block, 0, s, a, z); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T, typename U>
hipError_t launch_ytri(int M, int K, const YArgs<T, U>& a, const ZeroArgs& z, hipStream_t s) {
  const long nb = (a.Q + M - 1) / M + 1;   // + the (0,0)-mode block
  dim3 grid((unsigned)nb);
  switch (M) {
    case 16: return launch_ytri_m<T, U, 16>(K, a, z, s, grid);
    case 8: return launch_ytri_m<T, U, 8>(K, a, z, s, grid);
    case 4: return launch_ytri_m<T, U, 4>(K, a, z, s, grid);
    default: return hipErrorInvalidValue;
  }
}

template hipError_t launch_ytri<double, double>(int, int, const YArgs<double, double>&, const ZeroArgs&, hipStream_t);
template hipError_t launch_ytri<float, float>(int, int, const YArgs<float, float>&, const ZeroArgs&, hipStream_t);
template hipError_t launch_ytri<float, double>(int, int, const YArgs<float, double>&, const ZeroArgs&, hipStream_t);

}  // namespace ibp

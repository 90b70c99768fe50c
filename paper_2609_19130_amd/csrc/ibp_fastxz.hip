// Transforms along x and z for power-of-two lengths 32..1024, with the FFT
// held in registers (ibp_regfft.hpp).  Same contract as the generic LDS
// kernels of ibp_xz.hip (same layouts, partials, row sums and modes); the
// host picks these whenever nx/2 or nz is one of the supported lengths.
//
// x pass: TT = H/8 consecutive threads own one row; thread t loads the
// complex pairs (x[2m], x[2m+1]) for m = t + TT*i (16-byte accesses,
// consecutive threads on consecutive pairs), transforms, and writes the
// half-spectrum coefficients k = t + TT*i (+ k = H from thread 0).
// z pass: C consecutive threads own C consecutive kx columns of one y plane
// (C*element-size contiguous bytes per z), TT = NZ/8 thread groups cover z.
#include <cstdlib>

#include "ibp_internal.hpp"
#include "ibp_regfft.hpp"

namespace ibp {

using rfft::final_index;
using rfft::kE;
using rfft::pad8;

// x R2C of rows [blk*RB, blk*RB + RB) with NT threads (RB = NT / (H/8)).
// Every thread of the block must call it; it returns with LDS free.  PRE:
// the thread's eight input pairs were loaded beforehand into pre[0..8).
template <typename T, int MODE, int H, int NT, bool PRE = false>
__device__ __forceinline__ void xr2c_body(const XArgs<T>& A, long blk, Cx<T>* lds, double* sh, int tid,
                                          const double2* pre = nullptr) {
  constexpr int TT = H / kE;
  constexpr int SS = rfft::Seq<H>::stride;
  using P = rfft::Plan<H, false, T>;
  constexpr int RL = P::last_radix();
  constexpr int RB = NT / TT;
  const int lr = tid / TT, t = tid % TT;
  const long row = blk * RB + lr;
  const bool live = row < A.nrows;
  const int nx = A.nx, nz = A.nz, ny = A.ny;
  const int j = live ? (int)(row / nz) : 0;
  const int k = live ? (int)(row - (long)j * nz) : 0;
  constexpr bool kRes = MODE == XM_RESID || MODE == XM_RESID_ONLY;
  // norm partials: residual passes and FP32-spectrum passes (the mixed forms'
  // first pass); an FP64-spectrum right-hand-side pass (the direct solve)
  // never needs them and carries none of their registers
  constexpr bool kParts = kRes || sizeof(T) == 4;
  double mean = 0.0, s = 1.0;
  if (kRes) mean = A.ctl->removed_mean;
  if (MODE == XM_RESID) s = A.ctl->scale[A.iter & 1];

  Cx<T> v[kE];
  double rs = 0.0;
  NormAcc acc;
  const double dyfj = kRes && live ? A.dyf[j] : 0.0;
#pragma unroll
  for (int i = 0; i < kE; ++i) {
    const int m = t + TT * i;
    double v0 = 0.0, v1 = 0.0;
    if (live) {
      const double2 fv = PRE ? pre[i]
                         : MODE == XM_DIV ? assemble_pair(A, row, j, k, m)
                                          : *reinterpret_cast<const double2*>(A.f + row * nx + 2 * m);
      if (!kRes) {
        v0 = fv.x;
        v1 = fv.y;
        if (kParts && A.parts) acc.rhs_pair(v0, v1);
      } else {
        const double* prow = A.phi + row * nx;
        const double2 pc = *reinterpret_cast<const double2*>(prow + 2 * m);
        const double pl = prow[m == 0 ? nx - 1 : 2 * m - 1];
        const double pr = prow[2 * m + 2 == nx ? 0 : 2 * m + 2];
        const int kp = k + 1 == nz ? 0 : k + 1, km = k == 0 ? nz - 1 : k - 1;
        const double2 zp = *reinterpret_cast<const double2*>(A.phi + ((long)j * nz + kp) * nx + 2 * m);
        const double2 zm = *reinterpret_cast<const double2*>(A.phi + ((long)j * nz + km) * nx + 2 * m);
        double2 yp = make_double2(0.0, 0.0), ym = make_double2(0.0, 0.0);
        if (j + 1 < ny) yp = *reinterpret_cast<const double2*>(A.phi + ((long)(j + 1) * nz + k) * nx + 2 * m);
        if (j > 0) ym = *reinterpret_cast<const double2*>(A.phi + ((long)(j - 1) * nz + k) * nx + 2 * m);
        const double ca = A.ya[j], cc = A.yc[j];
        const double L0 = (pc.y - 2.0 * pc.x + pl) * A.idx2 + (zp.x + zm.x - 2.0 * pc.x) * A.idz2 +
                          ca * (ym.x - pc.x) + cc * (yp.x - pc.x);
        const double L1 = (pr - 2.0 * pc.y + pc.x) * A.idx2 + (zp.y + zm.y - 2.0 * pc.y) * A.idz2 +
                          ca * (ym.y - pc.y) + cc * (yp.y - pc.y);
        const double f0 = fv.x - mean, f1 = fv.y - mean;
        v0 = f0 - L0;
        v1 = f1 - L1;
        acc.pair(v0, v1, f0, f1, dyfj * dyfj);
        acc.phi_pair(pc.x, pc.y, dyfj);
      }
      rs += v0 + v1;
    }
    v[i] = Cx<T>{T(v0 * s), T(v1 * s)};
  }
  // FP64 row sum over the TT threads of the row (aligned power-of-two lane group)
#pragma unroll
  for (int off = TT / 2; off > 0; off >>= 1) rs += __shfl_xor(rs, off, kWave);
  if (live && t == 0) A.rowsum[row] = rs;
  if (kParts && A.parts) acc.write<NT, kRes>(A.part, blk, sh);
  Cx<T>* my = lds + lr * SS;
  P::run(v, t, my, A.twx, 2);
#pragma unroll
  for (int q = 0; q < kE; ++q) my[pad8(t + TT * final_index<RL>(q))] = v[q];
  __syncthreads();
  Cx<T>* srow = A.spec + row * A.rs + (row / nz) * (A.ps - (long)nz * A.rs);
#pragma unroll
  for (int i = 0; i < kE && live; ++i) {
    const int kk = t + TT * i;
    const Cx<T> Zk = my[pad8(kk)];
    const Cx<T> Zc = cconj(my[pad8((H - kk) & (H - 1))]);
    const Cx<T> E = cscale(cadd(Zk, Zc), T(0.5));
    const Cx<T> D = csub(Zk, Zc);
    const Cx<T> O = Cx<T>{T(0.5) * D.y, T(-0.5) * D.x};   // D / 2i
    const Cx<T> WO = cmul(A.twx[kk], O);
    srow[kk] = cadd(E, WO);
    if (kk == 0) srow[H] = cconj(csub(E, WO));
  }
  __syncthreads();
}

template <typename T, int MODE, int H>
__global__ __launch_bounds__(kThreads) void k_xr2c_reg(XArgs<T> A) {
  constexpr int RB = kThreads / (H / kE);
  __shared__ Cx<T> lds[RB * rfft::Seq<H>::stride];
  __shared__ double sh[(kThreads / kWave) * kPartStride];
  if ((MODE == XM_RESID || MODE == XM_RESID_ONLY) && A.ctl->done) return;
  if (MODE == XM_RESID_ONLY && A.probe && !A.ctl->probe) return;
  xr2c_body<T, MODE, H, kThreads>(A, A.row_begin / RB + blockIdx.x, lds, sh, threadIdx.x);
}

// Two row groups per block (plain right-hand side): the loads of both are
// issued before the first transform, so one group's memory traffic overlaps
// the other's transform (the single-group kernel leaves the FFT latency
// exposed: 0.42 ms against 0.35 ms for the 512x384x512 FP64 pass).
constexpr int kXGroups = 2;

template <typename T, int MODE, int H>
__global__ __launch_bounds__(kThreads) void k_xr2c_pipe(XArgs<T> A) {
  constexpr int TT = H / kE;
  constexpr int RB = kThreads / TT;
  __shared__ Cx<T> lds[RB * rfft::Seq<H>::stride];
  __shared__ double sh[(kThreads / kWave) * kPartStride];
  const long blk0 = A.row_begin / RB + (long)blockIdx.x * kXGroups;
  const int tid = threadIdx.x, lr = tid / TT, t = tid % TT;
  double2 buf[kXGroups][kE];
#pragma unroll
  for (int g = 0; g < kXGroups; ++g) {
    const long row = (blk0 + g) * RB + lr;
#pragma unroll
    for (int i = 0; i < kE; ++i)
      buf[g][i] = row < A.nrows ? *reinterpret_cast<const double2*>(A.f + row * A.nx + 2 * (t + TT * i))
                                : make_double2(0.0, 0.0);
  }
#pragma unroll
  for (int g = 0; g < kXGroups; ++g) xr2c_body<T, MODE, H, kThreads, true>(A, blk0 + g, lds, sh, tid, buf[g]);
}

// x C2R of rows [blk*RB, blk*RB + RB) with NT threads; called by every thread.
// PRE: the thread's spectrum pairs (X[k], X[H-k]) were loaded beforehand.
template <typename T, int MODE, int H, int NT, bool PRE = false>
__device__ __forceinline__ void xc2r_body(const XArgs<T>& A, long blk, Cx<T>* lds, int tid,
                                          const Cx<T>* pre = nullptr) {
  constexpr int TT = H / kE;
  constexpr int SS = rfft::Seq<H>::stride;
  using P = rfft::Plan<H, true, T>;
  constexpr int RL = P::last_radix();
  constexpr int RB = NT / TT;
  const int lr = tid / TT, t = tid % TT;
  const long row = blk * RB + lr;
  const bool live = row < A.nrows;
  Cx<T> v[kE];
  const long srow0 = live ? row * A.rs + (row / A.nz) * (A.ps - (long)A.nz * A.rs) : 0;
  const Cx<T>* srow = A.spec + srow0;
#pragma unroll
  for (int i = 0; i < kE; ++i) {
    const int kk = t + TT * i;
    Cx<T> Xk{T(0), T(0)}, Xm{T(0), T(0)};
    if (PRE) {
      Xk = pre[2 * i];
      Xm = pre[2 * i + 1];
    } else if (live) {
      Xk = srow[kk];
      Xm = srow[H - kk];
    }
    if (kk == 0) {
      Xk.y = T(0);
      Xm.y = T(0);
    }
    const Cx<T> Xmc = cconj(Xm);
    const Cx<T> E = cscale(cadd(Xk, Xmc), T(0.5));
    const Cx<T> D = cscale(csub(Xk, Xmc), T(0.5));
    const Cx<T> O = cmul(cconj(A.twx[kk]), D);
    v[i] = Cx<T>{E.x - O.y, E.y + O.x};   // E + i O
  }
  P::run(v, t, lds + lr * SS, A.twx, 2);
  if (!live) return;   // no barrier follows
  double cs = A.out_scale;
  if (MODE == CM_ADD) cs = cs / A.ctl->scale[A.iter & 1];
  const int j = (int)(row / A.nz);
  double c00 = A.phi00[j] * A.inv_nxnz;
  if (MODE == CM_ADD) c00 -= A.ctl->phimean;   // keep the iterate's weighted mean at zero
  double* orow = A.out + row * A.nx;
#pragma unroll
  for (int q = 0; q < kE; ++q) {
    const int m = t + TT * final_index<RL>(q);
    double v0 = double(v[q].x) * cs + c00, v1 = double(v[q].y) * cs + c00;
    double2* o = reinterpret_cast<double2*>(orow + 2 * m);
    if (MODE == CM_ADD) {
      const double2 old = *o;
      v0 += old.x;
      v1 += old.y;
    }
    *o = make_double2(v0, v1);
  }
}

template <typename T, int MODE, int H>
__global__ __launch_bounds__(kThreads) void k_xc2r_pipe(XArgs<T> A) {
  constexpr int TT = H / kE;
  constexpr int RB = kThreads / TT;
  __shared__ Cx<T> lds[RB * rfft::Seq<H>::stride];
  if (MODE == CM_ADD && A.ctl->done) return;
  const long blk0 = A.row_begin / RB + (long)rev_block_x() * kXGroups;
  const int tid = threadIdx.x, lr = tid / TT, t = tid % TT;
  Cx<T> buf[kXGroups][2 * kE];
#pragma unroll
  for (int g = 0; g < kXGroups; ++g) {
    const long row = (blk0 + g) * RB + lr;
    const bool live = row < A.nrows;
    const Cx<T>* srow = A.spec + (live ? row * A.rs + (row / A.nz) * (A.ps - (long)A.nz * A.rs) : 0);
#pragma unroll
    for (int i = 0; i < kE; ++i) {
      const int kk = t + TT * i;
      buf[g][2 * i] = live ? srow[kk] : Cx<T>{T(0), T(0)};
      buf[g][2 * i + 1] = live ? srow[H - kk] : Cx<T>{T(0), T(0)};
    }
  }
#pragma unroll
  for (int g = 0; g < kXGroups; ++g) {
    xc2r_body<T, MODE, H, kThreads, true>(A, blk0 + g, lds, tid, buf[g]);
    __syncthreads();   // the next group reuses the LDS rows
  }
}

template <typename T, int MODE, int H>
__global__ __launch_bounds__(kThreads) void k_xc2r_reg(XArgs<T> A) {
  constexpr int RB = kThreads / (H / kE);
  __shared__ Cx<T> lds[RB * rfft::Seq<H>::stride];
  if (MODE == CM_ADD && A.ctl->done) return;
  xc2r_body<T, MODE, H, kThreads>(A, A.row_begin / RB + rev_block_x(), lds, threadIdx.x);
}

// z FFT of kx columns [colblk*C, colblk*C + C) of one y plane with C*NZ/8
// threads; called by every thread; returns with LDS free.
template <typename T, bool INV, int NZ, int C>
__device__ __forceinline__ void zfft_body(const ZfArgs<T>& A, int colblk, long plane_index, Cx<T>* lds,
                                          int tid) {
  constexpr int TT = NZ / kE;
  constexpr int SS = rfft::col_stride<NZ, C, sizeof(Cx<T>)>();
  using P = rfft::Plan<NZ, INV, T>;
  constexpr int RL = P::last_radix();
  const int c = tid % C, t = tid / C;
  const int col = colblk * C + c;
  const bool live = col < A.hp;
  const long rs = A.rs;
  Cx<T>* plane = A.spec + (size_t)plane_index * A.ps;
  Cx<T> v[kE];
#pragma unroll
  for (int i = 0; i < kE; ++i) {
    const int z = t + TT * i;
    v[i] = live ? plane[(size_t)z * rs + col] : Cx<T>{T(0), T(0)};
  }
  P::run(v, t, lds + c * SS, A.twz, 1);
  if (!live) return;   // no barrier follows
#pragma unroll
  for (int q = 0; q < kE; ++q) {
    const int z = t + TT * final_index<RL>(q);
    plane[(size_t)z * rs + col] = v[q];
  }
}

template <typename T, bool INV, int NZ, int C>
__global__ __launch_bounds__(C*(NZ / kE)) void k_zfft_reg(ZfArgs<T> A) {
  __shared__ Cx<T> lds[C * rfft::col_stride<NZ, C, sizeof(Cx<T>)>()];
  if (A.check_done && A.ctl->done) return;
  // forward: planes in descending order (the x R2C wrote the last planes
  // last); inverse of an FP64 spectrum: grid (planes, column groups), column
  // groups in descending order (its line solve wrote the last kx groups last)
  if (INV && sizeof(T) == 8)
    zfft_body<T, INV, NZ, C>(A, rev_block_y(), A.plane0 + blockIdx.x, lds, threadIdx.x);
  else if (INV)
    zfft_body<T, INV, NZ, C>(A, blockIdx.x, A.plane0 + blockIdx.y, lds, threadIdx.x);
  else
    zfft_body<T, INV, NZ, C>(A, blockIdx.x, A.plane0 + rev_block_y(), lds, threadIdx.x);
}


// ---------------------------------------------------------------- FP64 inverse of an FP32 spectrum
// FP64 inverse z transform of kx columns [colblk C, colblk C + C) of plane
// j of the FP32 spectrum, written to the FP64 spectrum (the first step of
// the mixed form's direct first correction; ZupArgs).
template <int NZ, int C>
__global__ __launch_bounds__(C*(NZ / kE)) void k_zinv_up(ZupArgs A) {
  constexpr int TT = NZ / kE;
  constexpr int SS = rfft::col_stride<NZ, C, sizeof(Cx<double>)>();
  using P = rfft::Plan<NZ, true, double>;
  constexpr int RL = P::last_radix();
  __shared__ Cx<double> lds[C * SS];
  const int colblk = blockIdx.x, j = blockIdx.y;
  const int tid = threadIdx.x, c = tid % C, t = tid / C;
  const int col = colblk * C + c;
  const bool live = col < A.hp;
  const Cx<float>* in = A.in + (size_t)j * A.ips;
  Cx<double> v[kE];
#pragma unroll
  for (int i = 0; i < kE; ++i) {
    const int z = t + TT * i;
    const Cx<float> w = live ? in[(size_t)z * A.irs + col] : Cx<float>{0.0f, 0.0f};
    v[i] = Cx<double>{double(w.x), double(w.y)};
    if (A.zero00 && col == 0 && z == 0) v[i] = Cx<double>{0.0, 0.0};
  }
  P::run(v, t, lds + c * SS, A.twz, 1);
  if (!live) return;   // no barrier follows
  Cx<double>* out = A.out + (size_t)j * A.ops;
#pragma unroll
  for (int q = 0; q < kE; ++q) {
    const int z = t + TT * final_index<RL>(q);
    out[(size_t)z * A.ors + col] = v[q];
  }
}

// Per row: FP64 inverse x transform of the z-inverted FP64 spectrum, r0 =
// f - t - (plane mean), then the FP32 forward x transform of r0 * s into the
// FP32 half spectrum, with the row sums and norm partials of r0 (RtArgs).
template <int H>
__global__ __launch_bounds__(kThreads) void k_x_roundtrip(RtArgs R) {
  constexpr int TT = H / kE;
  constexpr int SS = rfft::Seq<H>::stride;
  constexpr int RB = kThreads / TT;
  using PI = rfft::Plan<H, true, double>;
  using PF = rfft::Plan<H, false, float>;
  constexpr int RLI = PI::last_radix();
  constexpr int RLF = PF::last_radix();
  __shared__ Cx<double> lds[RB * SS];
  __shared__ double sh[(kThreads / kWave) * kPartStride];
  const XArgs<float>& A = R.x;
  const int tid = threadIdx.x, lr = tid / TT, t = tid % TT;
  const long blk = blockIdx.x;
  const long row = blk * RB + lr;
  const bool live = row < A.nrows;
  const int nz = A.nz, nx = A.nx;
  const int j = live ? (int)(row / nz) : 0;
  // the row of f, loaded with the spectrum (pair m = t + TT i in fv[i])
  double2 fv[kE];
  {
    const double* frow = A.f + (live ? row : 0) * nx;
#pragma unroll
    for (int i = 0; i < kE; ++i)
      fv[i] = live ? *reinterpret_cast<const double2*>(frow + 2 * (t + TT * i)) : make_double2(0.0, 0.0);
  }
  // inverse x transform (FP64) of the row, as in the C2R pass
  Cx<double> v[kE];
  {
    const Cx<double>* trow = R.t64 + (live ? row * R.trs + (row / nz) * (R.tps - (long)nz * R.trs) : 0);
#pragma unroll
    for (int i = 0; i < kE; ++i) {
      const int kk = t + TT * i;
      Cx<double> Xk{0.0, 0.0}, Xm{0.0, 0.0};
      if (live) {
        Xk = trow[kk];
        Xm = trow[H - kk];
      }
      if (kk == 0) {
        Xk.y = 0.0;
        Xm.y = 0.0;
      }
      const Cx<double> Xmc = cconj(Xm);
      const Cx<double> E = cscale(cadd(Xk, Xmc), 0.5);
      const Cx<double> D = cscale(csub(Xk, Xmc), 0.5);
      const Cx<double> O = cmul(cconj(R.twx64[kk]), D);
      v[i] = Cx<double>{E.x - O.y, E.y + O.x};
    }
  }
  PI::run(v, t, lds + lr * SS, R.twx64, 2);
  __syncthreads();   // the FP32 transform below reuses the LDS rows
  const double cs = A.out_scale;
  const double pmean = (R.sub_mean && live) ? R.ghat[j] * A.inv_nxnz : 0.0;
  const double mean = A.ctl->removed_mean;
  const double s = A.ctl->scale[A.iter & 1];
  const double dyfj = live ? A.dyf[j] : 0.0;
  Cx<float> w[kE];
  double rs = 0.0;
  NormAcc acc;
#pragma unroll
  for (int q = 0; q < kE; ++q) {
    const int i = final_index<RLI>(q);   // inverse output q is pair m = t + TT i
    double r0 = 0.0, r1 = 0.0;
    if (live) {
      const double2 f = fv[i];
      r0 = f.x - v[q].x * cs - pmean;
      r1 = f.y - v[q].y * cs - pmean;
      acc.pair(r0, r1, f.x - mean, f.y - mean, dyfj * dyfj);
      rs += r0 + r1;
    }
    w[i] = Cx<float>{float(r0 * s), float(r1 * s)};
  }
#pragma unroll
  for (int off = TT / 2; off > 0; off >>= 1) rs += __shfl_xor(rs, off, kWave);
  if (live && t == 0) A.rowsum[row] = rs;
  acc.write<kThreads, true>(A.part, blk, sh);
  // forward x transform (FP32) of r0 * s, as in the R2C pass
  Cx<float>* my = reinterpret_cast<Cx<float>*>(lds) + lr * SS;
  PF::run(w, t, my, A.twx, 2);
#pragma unroll
  for (int q = 0; q < kE; ++q) my[pad8(t + TT * final_index<RLF>(q))] = w[q];
  __syncthreads();
  Cx<float>* srow = A.spec + row * A.rs + (row / nz) * (A.ps - (long)nz * A.rs);
#pragma unroll
  for (int i = 0; i < kE && live; ++i) {
    const int kk = t + TT * i;
    const Cx<float> Zk = my[pad8(kk)];
    const Cx<float> Zc = cconj(my[pad8((H - kk) & (H - 1))]);
    const Cx<float> E = cscale(cadd(Zk, Zc), 0.5f);
    const Cx<float> D = csub(Zk, Zc);
    const Cx<float> O = Cx<float>{0.5f * D.y, -0.5f * D.x};   // D / 2i
    const Cx<float> WO = cmul(A.twx[kk], O);
    srow[kk] = cadd(E, WO);
    if (kk == 0) srow[H] = cconj(csub(E, WO));
  }
}

hipError_t launch_zinv_up(const ZupArgs& a, hipStream_t s) {
  // 16 columns per block (64-byte FP32 input segments measured 7% slower
  // than the 128-byte ones of 16 columns), 8 for 1024-point lines (LDS)
  auto go = [&](auto kern, int nz, int C) {
    if (C * (nz / kE) > 1024) return hipErrorInvalidValue;
    const dim3 grid((unsigned)((a.hp + C - 1) / C), (unsigned)a.ny);
    hipLaunchKernelGGL(kern, grid, dim3(C * (nz / kE)), 0, s, a);
    return hipGetLastError();
  };
  switch (a.nz) {
    case 32: return go(k_zinv_up<32, 16>, 32, 16);
    case 64: return go(k_zinv_up<64, 16>, 64, 16);
    case 128: return go(k_zinv_up<128, 16>, 128, 16);
    case 256: return go(k_zinv_up<256, 16>, 256, 16);
    case 512: return go(k_zinv_up<512, 16>, 512, 16);
    case 1024: return go(k_zinv_up<1024, 8>, 1024, 8);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_x_roundtrip(const RtArgs& a, hipStream_t s) {
  auto go = [&](auto kern, int H) {
    const int RB = kThreads / (H / kE);
    const long nb = (a.x.nrows + RB - 1) / RB;
    hipLaunchKernelGGL(kern, dim3((unsigned)nb), dim3(kThreads), 0, s, a);
    return hipGetLastError();
  };
  switch (a.x.h) {
    case 32: return go(k_x_roundtrip<32>, 32);
    case 64: return go(k_x_roundtrip<64>, 64);
    case 128: return go(k_x_roundtrip<128>, 128);
    case 256: return go(k_x_roundtrip<256>, 256);
    case 512: return go(k_x_roundtrip<512>, 512);
    default: return hipErrorInvalidValue;
  }
}

// ---------------------------------------------------------------- fused x/z
// Item g of the round sequence -> (stage, plane, index within the plane).
__device__ __forceinline__ void decode_item(long g, int ny, int D, int n1, int n2, int* stage, int* plane,
                                            int* idx) {
  const long a = (long)D * n1;
  if (g < a) {
    *stage = 0;
    *plane = (int)(g / n1);
    *idx = (int)(g - (long)(*plane) * n1);
    return;
  }
  g -= a;
  const long n12 = (long)n1 + n2;
  const long b = (long)(ny - D) * n12;
  if (g < b) {
    const long r = g / n12;
    const int o = (int)(g - r * n12);
    if (o < n1) {
      *stage = 0;
      *plane = D + (int)r;
      *idx = o;
    } else {
      *stage = 1;
      *plane = (int)r;
      *idx = o - n1;
    }
    return;
  }
  g -= b;
  *stage = 1;
  *plane = (ny - D) + (int)(g / n2);
  *idx = (int)(g % n2);
}

// Control flow of the fused kernel is kept wave-uniform: the queue claim,
// the dependency wait and the completion count are done by all 64 lanes of
// wave 0 (only lane 0 adds 1) and their results are broadcast with
// readfirstlane.  With per-thread branches (threadIdx.x == 0) around these
// steps the compiler may thread the branches across the loop's barriers so
// that the other lanes loop back before lane 0 has claimed the next item.

__global__ void k_xcc_probe(int* out) {
  const int x = xcc_id();
  if (threadIdx.x == 0) out[blockIdx.x] = x;
}

hipError_t launch_xcc_probe(int* out, int nblocks, hipStream_t s) {
  hipLaunchKernelGGL(k_xcc_probe, dim3((unsigned)nblocks), dim3(64), 0, s, out);
  return hipGetLastError();
}

// Planes of queue q: q, q + nq, q + 2 nq, ... below ny.
__device__ __forceinline__ int queue_planes(int q, int nq, int ny) { return q < ny ? (ny - q + nq - 1) / nq : 0; }

// Coherence within one XCD: the vector L1 is write-through and the L2 is
// shared by all compute units of the XCD, so a producer's stores are in the
// L2 once its store counter drains (workgroup release), and a consumer reads
// them through the L2.  A consumer's L1 never holds an older copy of a line
// it reads: within one launch a block reads a line of the intermediate only
// after the line is final (forward) or only lines it wrote itself before
// (inverse z stage), and the L1 starts the launch empty.
template <typename T, int H, int NZ, bool FWD, int MODE>
__global__ __launch_bounds__(kFusedThreads) __attribute__((amdgpu_waves_per_eu(4))) void k_fused_xz(FusedArgs<T> F) {
  constexpr int NT = kFusedThreads;
  constexpr int RBX = NT / (H / kE), CZ = NT / (NZ / kE);
  constexpr int LX = RBX * rfft::Seq<H>::stride, LZ = CZ * rfft::col_stride<NZ, CZ, sizeof(Cx<T>)>();
  __shared__ Cx<T> lds[LX > LZ ? LX : LZ];
  __shared__ double sh[(NT / kWave) * kPartStride];
  __shared__ int item;
  const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x) / kWave;   // uniform
  const int lane = (int)threadIdx.x % kWave;
  if (FWD ? MODE != XM_PLAIN : MODE == CM_ADD) {
    if (__builtin_amdgcn_readfirstlane(F.x.ctl->done)) return;   // every block: no counter touched
  }
  const int q = __builtin_amdgcn_readfirstlane((int)F.xcc_queue[xcc_id()]);
  const int n12 = F.nfirst + F.nsecond;
  const int nplanes = q >= 0 ? queue_planes(q, F.nq, F.ny) : 0;
  const int lag = F.lag < nplanes ? F.lag : nplanes;
  const long total = (long)nplanes * n12;
  int* queue = F.queue + (q >= 0 ? q : 0);
  for (;;) {
    if (total == 0) break;
    if (wave == 0) {
      const int got = atomicAdd(queue, lane == 0 ? 1 : 0);
      item = __builtin_amdgcn_readfirstlane(got);
    }
    __syncthreads();
    const long g = __builtin_amdgcn_readfirstlane(item);
    __syncthreads();
    if (g >= total) break;
    int stage, k, idx;
    decode_item(g, nplanes, lag, F.nfirst, F.nsecond, &stage, &k, &idx);
    stage = __builtin_amdgcn_readfirstlane(stage);
    const int plane = __builtin_amdgcn_readfirstlane(q + k * F.nq);
    idx = __builtin_amdgcn_readfirstlane(idx);
    // Opaque copy of the thread index: keeps the bodies' per-thread index
    // arithmetic inside the loop instead of hoisted (and held in registers)
    // across both bodies.
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    if (stage == 0) {
      if (FWD)
        xr2c_body<T, MODE, H, NT>(F.x, (long)plane * F.nfirst + idx, lds, sh, tid);
      else
        zfft_body<T, true, NZ, CZ>(F.z, idx, plane, lds, tid);
      // wait until this wave's stores are acknowledged by the L2 (a workgroup
      // release fence emits no such wait: the waves of a block share the L1)
      __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
      __syncthreads();
      if (wave == 0) atomicAdd(&F.done[plane], lane == 0 ? 1 : 0);
    } else {
      if (wave == 0) wave_wait_count(&F.done[plane], F.nfirst, F.error);
      __syncthreads();
      if (FWD)
        zfft_body<T, false, NZ, CZ>(F.z, idx, plane, lds, tid);
      else
        xc2r_body<T, MODE, H, NT>(F.x, (long)plane * F.nsecond + idx, lds, tid);
      __syncthreads();
    }
  }
  if (wave == 0) {
    const int t = __builtin_amdgcn_readfirstlane(atomicAdd(F.exit_count, lane == 0 ? 1 : 0));
    if (t == (int)gridDim.x - 1) {   // every block has left its loop
      // a queue whose XCD received no block leaves its planes untransformed
      int unserved = 0;
      for (int qq = 0; qq < F.nq; ++qq) {
        const int claimed = __builtin_amdgcn_readfirstlane(
            __hip_atomic_load(F.queue + qq, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
        if (claimed < queue_planes(qq, F.nq, F.ny) * n12) unserved = 1;
      }
      if (unserved && lane == 0) __hip_atomic_store(F.error, 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      for (int j = lane; j < F.ny; j += kWave) F.done[j] = 0;
      if (lane < kMaxXcc) F.queue[lane] = 0;
      if (lane == 0) *F.exit_count = 0;
    }
  }
}

bool fused_supported(int h, int nz) {
  if (!rfft::supported(h) || !rfft::supported(nz) || nz != 2 * h) return false;
  return nz % fused_x_rows(h) == 0;
}
int fused_x_rows(int h) { return kFusedThreads / (h / kE); }
int fused_z_cols(int nz) { return kFusedThreads / (nz / kE); }

template <typename T>
hipError_t launch_fused_fwd(const FusedArgs<T>& a, int blocks, hipStream_t s) {
  const dim3 grid((unsigned)blocks), block(kFusedThreads);
  switch (a.x.h) {
    case 32: hipLaunchKernelGGL((k_fused_xz<T, 32, 64, true, XM_PLAIN>), grid, block, 0, s, a); break;
    case 64: hipLaunchKernelGGL((k_fused_xz<T, 64, 128, true, XM_PLAIN>), grid, block, 0, s, a); break;
    case 128: hipLaunchKernelGGL((k_fused_xz<T, 128, 256, true, XM_PLAIN>), grid, block, 0, s, a); break;
    case 256: hipLaunchKernelGGL((k_fused_xz<T, 256, 512, true, XM_PLAIN>), grid, block, 0, s, a); break;
    case 512: hipLaunchKernelGGL((k_fused_xz<T, 512, 1024, true, XM_PLAIN>), grid, block, 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T, int MODE>
static hipError_t fused_inv_m(const FusedArgs<T>& a, int blocks, hipStream_t s) {
  const dim3 grid((unsigned)blocks), block(kFusedThreads);
  switch (a.x.h) {
    case 32: hipLaunchKernelGGL((k_fused_xz<T, 32, 64, false, MODE>), grid, block, 0, s, a); break;
    case 64: hipLaunchKernelGGL((k_fused_xz<T, 64, 128, false, MODE>), grid, block, 0, s, a); break;
    case 128: hipLaunchKernelGGL((k_fused_xz<T, 128, 256, false, MODE>), grid, block, 0, s, a); break;
    case 256: hipLaunchKernelGGL((k_fused_xz<T, 256, 512, false, MODE>), grid, block, 0, s, a); break;
    case 512: hipLaunchKernelGGL((k_fused_xz<T, 512, 1024, false, MODE>), grid, block, 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_fused_inv(int cmode, const FusedArgs<T>& a, int blocks, hipStream_t s) {
  if (cmode == CM_SET) return fused_inv_m<T, CM_SET>(a, blocks, s);
  if constexpr (sizeof(T) == 4) {
    if (cmode == CM_ADD) return fused_inv_m<T, CM_ADD>(a, blocks, s);
  }
  return hipErrorInvalidValue;
}

template <typename T, int H>
static hipError_t fused_occ(int* blocks) {
  int a = 0, b = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
      &a, reinterpret_cast<const void*>(&k_fused_xz<T, H, 2 * H, true, XM_PLAIN>), kFusedThreads, 0);
  if (e == hipSuccess)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &b, reinterpret_cast<const void*>(&k_fused_xz<T, H, 2 * H, false, CM_SET>), kFusedThreads, 0);
  *blocks = a < b ? a : b;
  return e;
}

template <typename T>
hipError_t fused_blocks_per_cu(int h, int* blocks) {
  switch (h) {
    case 32: return fused_occ<T, 32>(blocks);
    case 64: return fused_occ<T, 64>(blocks);
    case 128: return fused_occ<T, 128>(blocks);
    case 256: return fused_occ<T, 256>(blocks);
    case 512: return fused_occ<T, 512>(blocks);
    default: *blocks = 0; return hipErrorInvalidValue;
  }
}
template hipError_t fused_blocks_per_cu<double>(int, int*);
template hipError_t fused_blocks_per_cu<float>(int, int*);

template hipError_t launch_fused_fwd<double>(const FusedArgs<double>&, int, hipStream_t);
template hipError_t launch_fused_fwd<float>(const FusedArgs<float>&, int, hipStream_t);
template hipError_t launch_fused_inv<double>(int, const FusedArgs<double>&, int, hipStream_t);
template hipError_t launch_fused_inv<float>(int, const FusedArgs<float>&, int, hipStream_t);

// ---------------------------------------------------------------- launchers
template <typename T, int MODE>
static hipError_t xr2c_h(int h, const XArgs<T>& a, hipStream_t s) {
  auto go = [&](auto kern, auto pipe, int H) {
    const int RB = kThreads / (H / kE);
    const long nb = (a.nrows - a.row_begin + RB - 1) / RB;
    if (MODE == XM_PLAIN && nb % kXGroups == 0)
      hipLaunchKernelGGL(pipe, dim3((unsigned)(nb / kXGroups)), dim3(kThreads), 0, s, a);
    else
      hipLaunchKernelGGL(kern, dim3((unsigned)nb), dim3(kThreads), 0, s, a);
    return hipGetLastError();
  };
  switch (h) {
    case 32: return go(k_xr2c_reg<T, MODE, 32>, k_xr2c_pipe<T, XM_PLAIN, 32>, 32);
    case 64: return go(k_xr2c_reg<T, MODE, 64>, k_xr2c_pipe<T, XM_PLAIN, 64>, 64);
    case 128: return go(k_xr2c_reg<T, MODE, 128>, k_xr2c_pipe<T, XM_PLAIN, 128>, 128);
    case 256: return go(k_xr2c_reg<T, MODE, 256>, k_xr2c_pipe<T, XM_PLAIN, 256>, 256);
    case 512: return go(k_xr2c_reg<T, MODE, 512>, k_xr2c_pipe<T, XM_PLAIN, 512>, 512);
    default: return hipErrorInvalidValue;
  }
}

template <typename T, int MODE>
static hipError_t xc2r_h(int h, const XArgs<T>& a, hipStream_t s) {
  auto go = [&](auto kern, auto pipe, int H) {
    const int RB = kThreads / (H / kE);
    const long nb = (a.nrows - a.row_begin + RB - 1) / RB;
    // FP32 only: two preloaded groups of FP64 spectrum pairs need ~200 VGPRs
    // (2 waves per SIMD) and measured slower than one group
    if (sizeof(T) == 4 && nb % kXGroups == 0)
      hipLaunchKernelGGL(pipe, dim3((unsigned)(nb / kXGroups)), dim3(kThreads), 0, s, a);
    else
      hipLaunchKernelGGL(kern, dim3((unsigned)nb), dim3(kThreads), 0, s, a);
    return hipGetLastError();
  };
  switch (h) {
    case 32: return go(k_xc2r_reg<T, MODE, 32>, k_xc2r_pipe<T, MODE, 32>, 32);
    case 64: return go(k_xc2r_reg<T, MODE, 64>, k_xc2r_pipe<T, MODE, 64>, 64);
    case 128: return go(k_xc2r_reg<T, MODE, 128>, k_xc2r_pipe<T, MODE, 128>, 128);
    case 256: return go(k_xc2r_reg<T, MODE, 256>, k_xc2r_pipe<T, MODE, 256>, 256);
    case 512: return go(k_xc2r_reg<T, MODE, 512>, k_xc2r_pipe<T, MODE, 512>, 512);
    default: return hipErrorInvalidValue;
  }
}

long fast_x_rows_per_block(int h) { return kThreads / (h / kE); }

template <typename T>
hipError_t launch_xr2c_fast(int mode, const XArgs<T>& a, hipStream_t s) {
  if (mode == XM_PLAIN) return xr2c_h<T, XM_PLAIN>(a.h, a, s);
  if (mode == XM_RESID) return xr2c_h<T, XM_RESID>(a.h, a, s);
  if constexpr (sizeof(T) == 8) {   // right-hand side assembled in the pass: FP64 direct solves
    if (mode == XM_DIV) return xr2c_h<T, XM_DIV>(a.h, a, s);
  }
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_xc2r_fast(int mode, const XArgs<T>& a, hipStream_t s) {
  if (mode == CM_SET) return xc2r_h<T, CM_SET>(a.h, a, s);
  if (mode == CM_ADD) return xc2r_h<T, CM_ADD>(a.h, a, s);
  return hipErrorInvalidValue;
}

// kx columns per z-pass block: 128-byte segments where the block fits 1024 threads
template <typename T>
int fast_z_cols(int nz) {
  const int seg = 128 / (int)sizeof(Cx<T>);
  const int maxc = 1024 / (nz / kE);
  return seg < maxc ? seg : maxc;
}

template <typename T, bool INV>
static hipError_t zfft_n(const ZfArgs<T>& a, int nplanes, hipStream_t s) {
  const int C = fast_z_cols<T>(a.nz);
  // (two planes per block with both loaded up front was measured slower: the
  // preloaded columns double the VGPRs and halve the occupancy)
  const unsigned ncb = (unsigned)((a.hp + C - 1) / C);
  const dim3 grid = (INV && sizeof(T) == 8) ? dim3((unsigned)nplanes, ncb) : dim3(ncb, (unsigned)nplanes);
  auto go = [&](auto kern, int threads) {
    hipLaunchKernelGGL(kern, grid, dim3(threads), 0, s, a);
    return hipGetLastError();
  };
  constexpr int S = 128 / (int)sizeof(Cx<T>);   // 8 (FP64) or 16 (FP32)
  switch (a.nz) {
    case 32: return go(k_zfft_reg<T, INV, 32, S>, S * 4);
    case 64: return go(k_zfft_reg<T, INV, 64, S>, S * 8);
    case 128: return go(k_zfft_reg<T, INV, 128, S>, S * 16);
    case 256: return go(k_zfft_reg<T, INV, 256, S>, S * 32);
    case 512: return go(k_zfft_reg<T, INV, 512, S>, S * 64);
    case 1024: return go(k_zfft_reg<T, INV, 1024, 1024 / 128>, 1024);
    default: return hipErrorInvalidValue;
  }
}

template <typename T>
hipError_t launch_zfft_fast(bool inverse, const ZfArgs<T>& a, int nplanes, hipStream_t s) {
  return inverse ? zfft_n<T, true>(a, nplanes, s) : zfft_n<T, false>(a, nplanes, s);
}

template hipError_t launch_xr2c_fast<double>(int, const XArgs<double>&, hipStream_t);
template hipError_t launch_xr2c_fast<float>(int, const XArgs<float>&, hipStream_t);
template hipError_t launch_xc2r_fast<double>(int, const XArgs<double>&, hipStream_t);
template hipError_t launch_xc2r_fast<float>(int, const XArgs<float>&, hipStream_t);
template hipError_t launch_zfft_fast<double>(bool, const ZfArgs<double>&, int, hipStream_t);
template hipError_t launch_zfft_fast<float>(bool, const ZfArgs<float>&, int, hipStream_t);
template int fast_z_cols<double>(int);
template int fast_z_cols<float>(int);

}  // namespace ibp

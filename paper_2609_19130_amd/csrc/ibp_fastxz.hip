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
#include "ibp_internal.hpp"
#include "ibp_regfft.hpp"

namespace ibp {

using rfft::final_index;
using rfft::kE;
using rfft::pad8;

template <typename T, int MODE, int H>
__global__ __launch_bounds__(kThreads) void k_xr2c_reg(XArgs<T> A) {
  constexpr int TT = H / kE;
  constexpr int RB = kThreads / TT;
  constexpr int SS = rfft::Seq<H>::stride;
  using P = rfft::Plan<H, false, T>;
  constexpr int RL = P::last_radix();
  __shared__ Cx<T> lds[RB * SS];
  __shared__ double sh[4 * 5];
  if (MODE != XM_PLAIN && A.ctl->done) return;
  const int lr = threadIdx.x / TT, t = threadIdx.x % TT;
  const long blk = A.row_begin / RB + blockIdx.x;
  const long row = blk * RB + lr;
  const bool live = row < A.nrows;
  const int nx = A.nx, nz = A.nz, ny = A.ny;
  const int j = live ? (int)(row / nz) : 0;
  const int k = live ? (int)(row - (long)j * nz) : 0;
  double mean = 0.0, s = 1.0;
  if (MODE != XM_PLAIN) mean = A.ctl->removed_mean;
  if (MODE == XM_RESID) s = A.ctl->scale[A.iter & 1];

  Cx<T> v[kE];
  double rs = 0.0, acc_in2 = 0.0, acc_f2 = 0.0, acc_max = 0.0, acc_bad = 0.0, acc_wphi = 0.0;
#pragma unroll
  for (int i = 0; i < kE; ++i) {
    const int m = t + TT * i;
    double v0 = 0.0, v1 = 0.0;
    if (live) {
      const double2 fv = *reinterpret_cast<const double2*>(A.f + row * nx + 2 * m);
      if (MODE == XM_PLAIN) {
        v0 = fv.x;
        v1 = fv.y;
        acc_f2 += v0 * v0 + v1 * v1;
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
        acc_f2 += f0 * f0 + f1 * f1;
        acc_wphi += A.dyf[j] * (pc.x + pc.y);
      }
      rs += v0 + v1;
      acc_in2 += v0 * v0 + v1 * v1;
      acc_max = fmax(acc_max, fmax(fabs(v0), fabs(v1)));
      if (!isfinite(v0) || !isfinite(v1)) acc_bad += 1.0;
    }
    v[i] = Cx<T>{T(v0 * s), T(v1 * s)};
  }
  // FP64 row sum over the TT threads of the row (aligned power-of-two lane group)
#pragma unroll
  for (int off = TT / 2; off > 0; off >>= 1) rs += __shfl_xor(rs, off, kWave);
  if (live && t == 0) A.rowsum[row] = rs;
  if (A.parts) {
    double vals[5] = {acc_in2, acc_f2, acc_max, acc_bad, acc_wphi};
    const bool ismax[5] = {false, false, true, false, false};
    block_reduce<5>(vals, ismax, sh);
    if (threadIdx.x == 0) {
#pragma unroll
      for (int q = 0; q < kPartStride; ++q) A.part[blk * kPartStride + q] = vals[q];
    }
  }
  Cx<T>* my = lds + lr * SS;
  P::run(v, t, my, A.twx, 2);
#pragma unroll
  for (int q = 0; q < kE; ++q) my[pad8(t + TT * final_index<RL>(q))] = v[q];
  __syncthreads();
  if (!live) return;
  Cx<T>* srow = A.spec + row * A.rs + (row / nz) * (A.ps - (long)nz * A.rs);
#pragma unroll
  for (int i = 0; i < kE; ++i) {
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
}

template <typename T, int MODE, int H>
__global__ __launch_bounds__(kThreads) void k_xc2r_reg(XArgs<T> A) {
  constexpr int TT = H / kE;
  constexpr int RB = kThreads / TT;
  constexpr int SS = rfft::Seq<H>::stride;
  using P = rfft::Plan<H, true, T>;
  constexpr int RL = P::last_radix();
  __shared__ Cx<T> lds[RB * SS];
  if (MODE == CM_ADD && A.ctl->done) return;
  const int lr = threadIdx.x / TT, t = threadIdx.x % TT;
  const long blk = A.row_begin / RB + blockIdx.x;
  const long row = blk * RB + lr;
  const bool live = row < A.nrows;
  Cx<T> v[kE];
  const long srow0 = live ? row * A.rs + (row / A.nz) * (A.ps - (long)A.nz * A.rs) : 0;
  const Cx<T>* srow = A.spec + srow0;
#pragma unroll
  for (int i = 0; i < kE; ++i) {
    const int kk = t + TT * i;
    Cx<T> Xk{T(0), T(0)}, Xm{T(0), T(0)};
    if (live) {
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
  if (!live) return;
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

template <typename T, bool INV, int NZ, int C>
__global__ __launch_bounds__(C*(NZ / kE)) void k_zfft_reg(ZfArgs<T> A) {
  constexpr int TT = NZ / kE;
  constexpr int SS = rfft::Seq<NZ>::stride;
  using P = rfft::Plan<NZ, INV, T>;
  constexpr int RL = P::last_radix();
  __shared__ Cx<T> lds[C * SS];
  if (A.check_done && A.ctl->done) return;
  const int c = threadIdx.x % C, t = threadIdx.x / C;
  const int col = blockIdx.x * C + c;
  const bool live = col < A.hp;
  const long rs = A.rs;
  Cx<T>* plane = A.spec + (size_t)(A.plane0 + blockIdx.y) * A.ps;
  Cx<T> v[kE];
#pragma unroll
  for (int i = 0; i < kE; ++i) {
    const int z = t + TT * i;
    v[i] = live ? plane[(size_t)z * rs + col] : Cx<T>{T(0), T(0)};
  }
  P::run(v, t, lds + c * SS, A.twz, 1);
  if (!live) return;
#pragma unroll
  for (int q = 0; q < kE; ++q) {
    const int z = t + TT * final_index<RL>(q);
    plane[(size_t)z * rs + col] = v[q];
  }
}

// ---------------------------------------------------------------- launchers
template <typename T, int MODE>
static hipError_t xr2c_h(int h, const XArgs<T>& a, hipStream_t s) {
  auto go = [&](auto kern, int H) {
    const int RB = kThreads / (H / kE);
    const long nb = (a.nrows - a.row_begin + RB - 1) / RB;
    hipLaunchKernelGGL(kern, dim3((unsigned)nb), dim3(kThreads), 0, s, a);
    return hipGetLastError();
  };
  switch (h) {
    case 32: return go(k_xr2c_reg<T, MODE, 32>, 32);
    case 64: return go(k_xr2c_reg<T, MODE, 64>, 64);
    case 128: return go(k_xr2c_reg<T, MODE, 128>, 128);
    case 256: return go(k_xr2c_reg<T, MODE, 256>, 256);
    case 512: return go(k_xr2c_reg<T, MODE, 512>, 512);
    default: return hipErrorInvalidValue;
  }
}

template <typename T, int MODE>
static hipError_t xc2r_h(int h, const XArgs<T>& a, hipStream_t s) {
  auto go = [&](auto kern, int H) {
    const int RB = kThreads / (H / kE);
    const long nb = (a.nrows - a.row_begin + RB - 1) / RB;
    hipLaunchKernelGGL(kern, dim3((unsigned)nb), dim3(kThreads), 0, s, a);
    return hipGetLastError();
  };
  switch (h) {
    case 32: return go(k_xc2r_reg<T, MODE, 32>, 32);
    case 64: return go(k_xc2r_reg<T, MODE, 64>, 64);
    case 128: return go(k_xc2r_reg<T, MODE, 128>, 128);
    case 256: return go(k_xc2r_reg<T, MODE, 256>, 256);
    case 512: return go(k_xc2r_reg<T, MODE, 512>, 512);
    default: return hipErrorInvalidValue;
  }
}

long fast_x_rows_per_block(int h) { return kThreads / (h / kE); }

template <typename T>
hipError_t launch_xr2c_fast(int mode, const XArgs<T>& a, hipStream_t s) {
  if (mode == XM_PLAIN) return xr2c_h<T, XM_PLAIN>(a.h, a, s);
  if (mode == XM_RESID) return xr2c_h<T, XM_RESID>(a.h, a, s);
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
  const dim3 grid((unsigned)((a.hp + C - 1) / C), (unsigned)nplanes);
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

// General (LDS, mixed-radix) transforms along the two periodic directions
// (paper: batched 2-D real FFTs on the x1-x2 planes diagonalise the periodic
// directions of the elliptic problem; "Fluid domain" parallelisation
// subsection).  Kernel templates shared by the two kernel families
// (ibp_xz.hip: every stage kind; ibp_xz_narrow.hip: radices 2, 3, 4, 5, 8).
//
// x pass: each row of nx reals is read as h = nx/2 complex pairs
// (x[2m], x[2m+1]), transformed by an h-point complex FFT in LDS, and split
// into the nx/2+1 half-spectrum coefficients X[k] = E[k] + W_nx^k O[k] with
// E = (Z[k] + conj Z[h-k]) / 2 and O = (Z[k] - conj Z[h-k]) / 2i.  The inverse
// reverses both steps.  A row of odd length (h = nx) is transformed as nx
// complex values (x[m], 0) and its first (nx+1)/2 coefficients are kept; the
// inverse rebuilds the other half as X[nx-k] = conj X[k].  One block owns
// `rows_per_block` whole rows; each wave loads whole rows with 16-byte
// coalesced accesses and sums them in FP64 for the (0,0) mode.
//
// z pass: one block owns one y plane and `cols` consecutive kx columns of
// the half spectrum; consecutive threads read consecutive kx (contiguous
// segments), the tile is transposed into LDS as one sequence per column and
// transformed along z, then written back in place.
#pragma once

#include "ibp_internal.hpp"

namespace ibp {

// Rows [blk * RB, blk * RB + RB) of one grid; every thread of the block calls
// it, and it returns with LDS free (uniform early exits only).
template <typename T, int MODE, int TILE, bool WIDE>
__device__ __forceinline__ void xr2c_gen_body(const XArgs<T>& A, const FftPlan& fp, long blk, Cx<T>* buf,
                                              double* sh) {
  constexpr bool kRes = MODE == XM_RESID || MODE == XM_RESID_ONLY;
  constexpr bool kParts = kRes || sizeof(T) == 4;   // as in the register kernels
  if (kRes && __builtin_amdgcn_readfirstlane(A.ctl->done)) return;
  if (MODE == XM_RESID_ONLY && A.probe && !__builtin_amdgcn_readfirstlane(A.ctl->probe)) return;
  const int h = A.h, RB = A.rows_per_block, nx = A.nx, nz = A.nz, ny = A.ny;
  const int hs = A.hs ? A.hs : h;   // LDS row stride (Bluestein: the convolution length)
  const bool odd = nx & 1;   // h = nx: single values, no split
  const long row0 = blk * RB;
  // row = j nz + k: the block's first row splits once, later rows by exact
  // small quotients (rows of a grid number below 2^31)
  const int j0 = (int)row0 / nz, k0 = (int)row0 - j0 * nz;
  const QDiv qnz = qdiv(nz);
  const long pgap = A.ps - (long)nz * A.rs;   // spectral plane padding
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  NormAcc acc;
  double mean = 0.0, s = 1.0;
  if (kRes) mean = A.ctl->removed_mean;
  if (MODE == XM_RESID) s = A.ctl->scale[A.iter & 1];

  for (int lr = wave; lr < RB; lr += kThreads / kWave) {
    const long row = row0 + lr;
    if (row >= A.nrows) {
      if (MODE != XM_RESID_ONLY)
        for (int m = lane; m < h; m += kWave) buf[lr * hs + m] = Cx<T>{T(0), T(0)};
      continue;
    }
    const IBP_GLOBAL double* frow = gbl(A.f) + row * nx;
    double rs = 0.0;
    const int jr = qquo(k0 + lr, qnz);
    const int j = j0 + jr;
    const int k = k0 + lr - __mul24(jr, nz);
    const double dyfj = kRes ? gbl(A.dyf)[j] : 0.0;
    if (odd) {
      for (int m = lane; m < nx; m += kWave) {
        const double fv = MODE == XM_DIV ? assemble_one(A, row, j, k, m) : frow[m];
        double v0;
        if (!kRes) {
          v0 = fv;
          if (kParts && A.parts) acc.rhs_one(v0);
        } else {
          // r = (f - m) - L_h phi, 7-point staggered stencil, FP64
          const IBP_GLOBAL double* prow = gbl(A.phi) + row * nx;
          const double pc = prow[m];
          const double pl = prow[m == 0 ? nx - 1 : m - 1];
          const double pr = prow[m + 1 == nx ? 0 : m + 1];
          const int kp = k + 1 == nz ? 0 : k + 1, km = k == 0 ? nz - 1 : k - 1;
          const double zp = gbl(A.phi)[((long)j * nz + kp) * nx + m];
          const double zm = gbl(A.phi)[((long)j * nz + km) * nx + m];
          const double yp = j + 1 < ny ? gbl(A.phi)[((long)(j + 1) * nz + k) * nx + m] : 0.0;
          const double ym = j > 0 ? gbl(A.phi)[((long)(j - 1) * nz + k) * nx + m] : 0.0;
          const double L0 = (pr - 2.0 * pc + pl) * A.idx2 + (zp + zm - 2.0 * pc) * A.idz2 + A.ya[j] * (ym - pc) +
                            A.yc[j] * (yp - pc);
          const double f0 = fv - mean;
          v0 = f0 - L0;
          acc.one(v0, f0, dyfj * dyfj);
          acc.phi_one(pc, dyfj);
        }
        rs += v0;
        if (MODE != XM_RESID_ONLY) buf[lr * hs + m] = Cx<T>{T(v0 * s), T(0)};
      }
    } else
    for (int m = lane; m < h; m += kWave) {
      const double2 fv = MODE == XM_DIV ? assemble_pair(A, row, j, k, m)
                                        : gld2(frow + 2 * m);
      double v0, v1;
      if (!kRes) {
        v0 = fv.x;
        v1 = fv.y;
        if (kParts && A.parts) acc.rhs_pair(v0, v1);
      } else {
        // r = (f - m) - L_h phi, 7-point staggered stencil, FP64
        const IBP_GLOBAL double* prow = gbl(A.phi) + row * nx;
        const double2 pc = gld2(prow + 2 * m);
        const double pl = prow[m == 0 ? nx - 1 : 2 * m - 1];
        const double pr = prow[2 * m + 2 == nx ? 0 : 2 * m + 2];
        const int kp = k + 1 == nz ? 0 : k + 1, km = k == 0 ? nz - 1 : k - 1;
        const double2 zp = gld2(gbl(A.phi) + ((long)j * nz + kp) * nx + 2 * m);
        const double2 zm = gld2(gbl(A.phi) + ((long)j * nz + km) * nx + 2 * m);
        double2 yp = make_double2(0.0, 0.0), ym = make_double2(0.0, 0.0);
        if (j + 1 < ny) yp = gld2(gbl(A.phi) + ((long)(j + 1) * nz + k) * nx + 2 * m);
        if (j > 0) ym = gld2(gbl(A.phi) + ((long)(j - 1) * nz + k) * nx + 2 * m);
        // y part as a difference of face fluxes (a_0 = c_{ny-1} = 0)
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
      if (MODE != XM_RESID_ONLY) buf[lr * hs + m] = Cx<T>{T(v0 * s), T(v1 * s)};
    }
    rs = wave_sum(rs);
    if (MODE != XM_RESID_ONLY && lane == 0) gbl(A.rowsum)[row] = rs;
  }
  if (kParts && A.parts) acc.write<kThreads, kRes>(gbl(A.part), blk, sh);
  if (MODE == XM_RESID_ONLY) return;
  __syncthreads();
  lds_fft<TILE, false, T, WIDE>(buf, RB, hs, fp, gbl(A.twx), odd ? 1 : 2, gbl(A.bc), gbl(A.bb), gbl(A.bt));

  if (odd) {   // the first (nx+1)/2 coefficients, no split
    const QDiv qhp = qdiv(A.hp);
    for (int e = threadIdx.x; e < RB * A.hp; e += kThreads) {
      const int lr = qquo(e, qhp), kk = e - __mul24(lr, A.hp);
      const long row = row0 + lr;
      if (row < A.nrows)
        gst(gbl(A.spec) + row * A.rs + (j0 + qquo(k0 + lr, qnz)) * pgap + kk, buf[__mul24(lr, hs) + kk]);
    }
    __syncthreads();
    return;
  }
  const int hh = h / 2 + 1;
  const QDiv qhh = qdiv(hh);
  for (int e = threadIdx.x; e < RB * hh; e += kThreads) {
    const int lr = qquo(e, qhh), k = e - __mul24(lr, hh);
    const long row = row0 + lr;
    if (row >= A.nrows) continue;
    const Cx<T> Zk = buf[__mul24(lr, hs) + k];   // k < hh <= h
    const Cx<T> Zc = cconj(buf[__mul24(lr, hs) + (k ? h - k : 0)]);
    const Cx<T> E = cscale(cadd(Zk, Zc), T(0.5));
    const Cx<T> D = csub(Zk, Zc);
    const Cx<T> O = Cx<T>{T(0.5) * D.y, T(-0.5) * D.x};     // D / 2i
    const Cx<T> WO = cmul(gld(gbl(A.twx) + k), O);
    IBP_GLOBAL Cx<T>* srow = gbl(A.spec) + row * A.rs + (j0 + qquo(k0 + lr, qnz)) * pgap;
    gst(srow + k, cadd(E, WO));
    if (h - k != k) gst(srow + (h - k), cconj(csub(E, WO)));
  }
  __syncthreads();
}

template <typename T, int MODE, int TILE, bool WIDE>
__global__ __launch_bounds__(kThreads) void k_xr2c(XArgs<T> A) {
  __shared__ Cx<T> buf[TILE];
  __shared__ double sh[4 * kPartStride];
  xr2c_gen_body<T, MODE, TILE, WIDE>(A, A.fp, A.row_begin / A.rows_per_block + blockIdx.x, buf, sh);
}

template <typename T, int MODE, int TILE, bool WIDE>
__device__ __forceinline__ void xc2r_gen_body(const XArgs<T>& A, const FftPlan& fp, long blk, Cx<T>* buf) {
  if (MODE == CM_ADD && __builtin_amdgcn_readfirstlane(A.ctl->done)) return;
  const int h = A.h, RB = A.rows_per_block, nx = A.nx, nz = A.nz;
  const int hs = A.hs ? A.hs : h;   // LDS row stride (Bluestein: the convolution length)
  const bool odd = nx & 1;   // h = nx: rebuild the full spectrum
  const long row0 = blk * RB;
  const int hh = odd ? 0 : h / 2 + 1;
  // row = j nz + k: the block's first row splits once, later rows by exact
  // small quotients (rows of a grid number below 2^31)
  const int j0 = (int)row0 / nz, k0 = (int)row0 - j0 * nz;
  const QDiv qnz = qdiv(nz);
  const long pgap = A.ps - (long)nz * A.rs;   // spectral plane padding
  if (odd) {
    const QDiv qhp = qdiv(A.hp);
    for (int e = threadIdx.x; e < RB * A.hp; e += kThreads) {
      const int lr = qquo(e, qhp), k = e - __mul24(lr, A.hp);
      const long row = row0 + lr;
      Cx<T> X{T(0), T(0)};
      if (row < A.nrows) X = gld(gbl(A.spec) + row * A.rs + (j0 + qquo(k0 + lr, qnz)) * pgap + k);
      if (k == 0) X.y = T(0);   // X[0] of a real sequence is real
      buf[__mul24(lr, hs) + k] = X;
      if (k > 0) buf[__mul24(lr, hs) + nx - k] = cconj(X);
    }
  }
  const QDiv qhh = qdiv(odd ? 1 : hh);
  for (int e = threadIdx.x; e < RB * hh; e += kThreads) {
    const int lr = qquo(e, qhh), k = e - __mul24(lr, hh);
    const long row = row0 + lr;
    Cx<T> Xk{T(0), T(0)}, Xm{T(0), T(0)};
    if (row < A.nrows) {
      const IBP_GLOBAL Cx<T>* srow = gbl(A.spec) + row * A.rs + (j0 + qquo(k0 + lr, qnz)) * pgap;
      Xk = gld(srow + k);
      Xm = gld(srow + (h - k));
    }
    if (k == 0) {           // X[0] and X[h] of a real sequence are real
      Xk.y = T(0);
      Xm.y = T(0);
    }
    const Cx<T> Xmc = cconj(Xm);
    const Cx<T> E = cscale(cadd(Xk, Xmc), T(0.5));
    const Cx<T> D = cscale(csub(Xk, Xmc), T(0.5));
    const Cx<T> O = cmul(cconj(gld(gbl(A.twx) + k)), D);
    buf[__mul24(lr, hs) + k] = Cx<T>{E.x - O.y, E.y + O.x};               // E + i O
    const int km = k ? h - k : 0;                                            // (h - k) mod h, k < hh <= h
    if (km != k) buf[__mul24(lr, hs) + km] = Cx<T>{E.x + O.y, O.x - E.y};   // conj(E) + i conj(O)
  }
  __syncthreads();
  lds_fft<TILE, true, T, WIDE>(buf, RB, hs, fp, gbl(A.twx), odd ? 1 : 2, gbl(A.bc), gbl(A.bb), gbl(A.bt));

  double cs = A.out_scale;
  if (MODE == CM_ADD) cs = cs / A.ctl->scale[A.iter & 1];
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  for (int lr = wave; lr < RB; lr += kThreads / kWave) {
    const long row = row0 + lr;
    if (row >= A.nrows) break;
    const int j = j0 + qquo(k0 + lr, qnz);
    double c00 = gbl(A.phi00)[j] * A.inv_nxnz;
    if (MODE == CM_ADD) c00 -= A.ctl->phimean;
    IBP_GLOBAL double* orow = gbl(A.out) + row * nx;
    if (odd) {
      for (int m = lane; m < nx; m += kWave) {
        double v0 = double(buf[lr * hs + m].x) * cs + c00;
        if (MODE == CM_ADD) v0 += orow[m];
        orow[m] = v0;
      }
      continue;
    }
    for (int m = lane; m < h; m += kWave) {
      const Cx<T> z = buf[lr * hs + m];
      double v0 = double(z.x) * cs + c00, v1 = double(z.y) * cs + c00;
      IBP_GLOBAL double* o = orow + 2 * m;
      if (MODE == CM_ADD) {
        const double2 old = gld2(o);
        v0 += old.x;
        v1 += old.y;
      }
      gst2(o, v0, v1);
    }
  }
  __syncthreads();
}

template <typename T, int MODE, int TILE, bool WIDE>
__global__ __launch_bounds__(kThreads) void k_xc2r(XArgs<T> A) {
  __shared__ Cx<T> buf[TILE];
  xc2r_gen_body<T, MODE, TILE, WIDE>(A, A.fp, A.row_begin / A.rows_per_block + rev_block_x(), buf);
}

template <typename T, bool INV, int TILE, bool WIDE>
__device__ __forceinline__ void zfft_gen_body(const ZfArgs<T>& A, const FftPlan& fp, int colblk, long plane_index,
                                              Cx<T>* buf) {
  if (A.check_done && __builtin_amdgcn_readfirstlane(A.ctl->done)) return;
  const int nz = A.nz, C = A.cols, hp = A.hp, ss = A.zss ? A.zss : nz + 1;
  const long rs = A.rs;
  const int c0 = colblk * C;
  IBP_GLOBAL Cx<T>* plane = gbl(A.spec) + (size_t)plane_index * A.ps;
  const QDiv qc = qdiv(C);
  for (int e = threadIdx.x; e < C * nz; e += kThreads) {
    const int z = qquo(e, qc), c = e - __mul24(z, C);
    buf[c * ss + z] = (c0 + c < hp) ? gld(plane + (size_t)z * rs + c0 + c) : Cx<T>{T(0), T(0)};
  }
  __syncthreads();
  lds_fft<TILE, INV, T, WIDE>(buf, C, ss, fp, gbl(A.twz), 1, gbl(A.bc), gbl(A.bb), gbl(A.bt));
  for (int e = threadIdx.x; e < C * nz; e += kThreads) {
    const int z = qquo(e, qc), c = e - __mul24(z, C);
    if (c0 + c < hp) gst(plane + (size_t)z * rs + c0 + c, buf[c * ss + z]);
  }
  __syncthreads();
}

template <typename T, bool INV, int TILE, bool WIDE>
__global__ __launch_bounds__(kThreads) void k_zfft(ZfArgs<T> A) {
  __shared__ Cx<T> buf[TILE + 64];
  zfft_gen_body<T, INV, TILE, WIDE>(A, A.fp, blockIdx.x, A.plane0 + (INV ? blockIdx.y : rev_block_y()), buf);
}

// ---------------------------------------------------------------- batched stages
// Per-grid arguments are copied from the device table into registers, except
// the FFT plans: the stage loops index them at run time, so they are read
// from the table in place (a private copy would live in scratch memory).
__device__ __forceinline__ int batch_grid_of(const long* start, int count, long b) {
  int lo = 0, hi = count - 1;   // largest g with start[g] <= b
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (__builtin_amdgcn_readfirstlane((int)(start[mid] <= b))) lo = mid; else hi = mid - 1;
  }
  return lo;
}

template <typename T, int MODE, int TILE, bool WIDE>
__global__ __launch_bounds__(kThreads) void kb_xr2c(const BatchGrid<T>* __restrict__ D, const long* __restrict__ start,
                                                     BatchPtrs P, BatchLaunch L) {
  __shared__ Cx<T> buf[TILE];
  __shared__ double sh[4 * kPartStride];
  const int g = batch_grid_of(start, L.count, blockIdx.x);
  XArgs<T> a = D[g].x;
  a.f = P.f[g];
  a.phi = P.phi[g];
  a.out = P.phi[g];
  a.iter = L.iter;
  xr2c_gen_body<T, MODE, TILE, WIDE>(a, D[g].x.fp, (long)blockIdx.x - start[g], buf, sh);
}

template <typename T, int MODE, int TILE, bool WIDE>
__global__ __launch_bounds__(kThreads) void kb_xc2r(const BatchGrid<T>* __restrict__ D, const long* __restrict__ start,
                                                     BatchPtrs P, BatchLaunch L) {
  __shared__ Cx<T> buf[TILE];
  const long bid = rev_block_x();
  const int g = batch_grid_of(start, L.count, bid);
  XArgs<T> a = D[g].x;
  a.f = P.f[g];
  a.phi = P.phi[g];
  a.out = P.phi[g];
  a.iter = L.iter;
  xc2r_gen_body<T, MODE, TILE, WIDE>(a, D[g].x.fp, bid - start[g], buf);
}

template <typename T, bool INV, int TILE, bool WIDE>
__global__ __launch_bounds__(kThreads) void kb_zfft(const BatchGrid<T>* __restrict__ D, const long* __restrict__ start,
                                                     BatchLaunch L) {
  __shared__ Cx<T> buf[TILE + 64];
  const long bid = INV ? blockIdx.x : rev_block_x();
  const int g = batch_grid_of(start, L.count, bid);
  ZfArgs<T> a = D[g].z;
  a.check_done = L.check_done;
  const long local = bid - start[g];
  const int ncb = D[g].zcolblocks;
  zfft_gen_body<T, INV, TILE, WIDE>(a, D[g].z.fp, (int)(local % ncb), local / ncb, buf);
}

// ---------------------------------------------------------------- launchers
// W selects the kernel family: with the radix-7/11, direct-sum and Bluestein
// stages (instantiated in ibp_xz.hip) or with radices 2, 3, 4, 5 and 8 only
// (ibp_xz_narrow.hip), which need far fewer registers.
template <typename T, bool W, int TL>
hipError_t batch_xr2c_tl(int mode, const BatchGrid<T>* d, const long* start, long nblocks, const BatchPtrs& p,
                         const BatchLaunch& l, hipStream_t s) {
  const dim3 grid((unsigned)nblocks), block(kThreads);
  switch (mode) {
    case XM_PLAIN: hipLaunchKernelGGL((kb_xr2c<T, XM_PLAIN, TL, W>), grid, block, 0, s, d, start, p, l); break;
    case XM_RESID: hipLaunchKernelGGL((kb_xr2c<T, XM_RESID, TL, W>), grid, block, 0, s, d, start, p, l); break;
    case XM_RESID_ONLY:
      hipLaunchKernelGGL((kb_xr2c<T, XM_RESID_ONLY, TL, W>), grid, block, 0, s, d, start, p, l);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T, bool W>
hipError_t batch_xr2c_w(int mode, bool small, const BatchGrid<T>* d, const long* start, long nblocks,
                        const BatchPtrs& p, const BatchLaunch& l, hipStream_t s) {
  if (small) return batch_xr2c_tl<T, W, sizeof(T) == 8 ? kTileX64s : kTileX32s>(mode, d, start, nblocks, p, l, s);
  return batch_xr2c_tl<T, W, sizeof(T) == 8 ? kTileX64 : kTileX32>(mode, d, start, nblocks, p, l, s);
}

template <typename T, bool W, int TL>
hipError_t batch_xc2r_tl(int mode, const BatchGrid<T>* d, const long* start, long nblocks, const BatchPtrs& p,
                         const BatchLaunch& l, hipStream_t s) {
  const dim3 grid((unsigned)nblocks), block(kThreads);
  switch (mode) {
    case CM_SET: hipLaunchKernelGGL((kb_xc2r<T, CM_SET, TL, W>), grid, block, 0, s, d, start, p, l); break;
    case CM_ADD: hipLaunchKernelGGL((kb_xc2r<T, CM_ADD, TL, W>), grid, block, 0, s, d, start, p, l); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T, bool W>
hipError_t batch_xc2r_w(int mode, bool small, const BatchGrid<T>* d, const long* start, long nblocks,
                        const BatchPtrs& p, const BatchLaunch& l, hipStream_t s) {
  if (small) return batch_xc2r_tl<T, W, sizeof(T) == 8 ? kTileX64s : kTileX32s>(mode, d, start, nblocks, p, l, s);
  return batch_xc2r_tl<T, W, sizeof(T) == 8 ? kTileX64 : kTileX32>(mode, d, start, nblocks, p, l, s);
}

template <typename T, bool W>
hipError_t batch_zfft_w(bool inverse, bool small, const BatchGrid<T>* d, const long* start, long nblocks,
                        const BatchLaunch& l, hipStream_t s) {
  constexpr int TL = (sizeof(T) == 8) ? kTileZ64 : kTileZ32;
  constexpr int TS = (sizeof(T) == 8) ? kTileZ64s : kTileZ32s;
  const dim3 grid((unsigned)nblocks), block(kThreads);
  if (small) {
    if (inverse)
      hipLaunchKernelGGL((kb_zfft<T, true, TS, W>), grid, block, 0, s, d, start, l);
    else
      hipLaunchKernelGGL((kb_zfft<T, false, TS, W>), grid, block, 0, s, d, start, l);
  } else {
    if (inverse)
      hipLaunchKernelGGL((kb_zfft<T, true, TL, W>), grid, block, 0, s, d, start, l);
    else
      hipLaunchKernelGGL((kb_zfft<T, false, TL, W>), grid, block, 0, s, d, start, l);
  }
  return hipGetLastError();
}

template <typename T, bool W, int TL>
hipError_t xr2c_tl(int mode, const XArgs<T>& a, hipStream_t s) {
  const long nblocks = (a.nrows - a.row_begin + a.rows_per_block - 1) / a.rows_per_block;
  dim3 grid((unsigned)nblocks), block(kThreads);
  switch (mode) {
    case XM_PLAIN: hipLaunchKernelGGL((k_xr2c<T, XM_PLAIN, TL, W>), grid, block, 0, s, a); break;
    case XM_RESID: hipLaunchKernelGGL((k_xr2c<T, XM_RESID, TL, W>), grid, block, 0, s, a); break;
    case XM_RESID_ONLY: hipLaunchKernelGGL((k_xr2c<T, XM_RESID_ONLY, TL, W>), grid, block, 0, s, a); break;
    case XM_DIV:
      if constexpr (sizeof(T) == 8) {
        hipLaunchKernelGGL((k_xr2c<T, XM_DIV, TL, W>), grid, block, 0, s, a);
        break;
      }
      return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T, bool W>
hipError_t xr2c_w(int mode, bool small, const XArgs<T>& a, hipStream_t s) {
  if (small) return xr2c_tl<T, W, sizeof(T) == 8 ? kTileX64s : kTileX32s>(mode, a, s);
  return xr2c_tl<T, W, sizeof(T) == 8 ? kTileX64 : kTileX32>(mode, a, s);
}

template <typename T, bool W, int TL>
hipError_t xc2r_tl(int mode, const XArgs<T>& a, hipStream_t s) {
  const long nblocks = (a.nrows - a.row_begin + a.rows_per_block - 1) / a.rows_per_block;
  dim3 grid((unsigned)nblocks), block(kThreads);
  switch (mode) {
    case CM_SET: hipLaunchKernelGGL((k_xc2r<T, CM_SET, TL, W>), grid, block, 0, s, a); break;
    case CM_ADD: hipLaunchKernelGGL((k_xc2r<T, CM_ADD, TL, W>), grid, block, 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T, bool W>
hipError_t xc2r_w(int mode, bool small, const XArgs<T>& a, hipStream_t s) {
  if (small) return xc2r_tl<T, W, sizeof(T) == 8 ? kTileX64s : kTileX32s>(mode, a, s);
  return xc2r_tl<T, W, sizeof(T) == 8 ? kTileX64 : kTileX32>(mode, a, s);
}

template <typename T, bool W>
hipError_t zfft_w(bool inverse, bool small, const ZfArgs<T>& a, int nplanes, hipStream_t s) {
  constexpr int TL = (sizeof(T) == 8) ? kTileZ64 : kTileZ32;
  constexpr int TS = (sizeof(T) == 8) ? kTileZ64s : kTileZ32s;
  dim3 grid((unsigned)((a.hp + a.cols - 1) / a.cols), (unsigned)nplanes), block(kThreads);
  if (small) {
    if (inverse)
      hipLaunchKernelGGL((k_zfft<T, true, TS, W>), grid, block, 0, s, a);
    else
      hipLaunchKernelGGL((k_zfft<T, false, TS, W>), grid, block, 0, s, a);
  } else {
    if (inverse)
      hipLaunchKernelGGL((k_zfft<T, true, TL, W>), grid, block, 0, s, a);
    else
      hipLaunchKernelGGL((k_zfft<T, false, TL, W>), grid, block, 0, s, a);
  }
  return hipGetLastError();
}

// Explicit instantiations of one family (PREFIX = extern: declarations only).
#define IBP_XZ_FAMILY(PREFIX, W)                                                                              \
  PREFIX template hipError_t xr2c_w<double, W>(int, bool, const XArgs<double>&, hipStream_t);                 \
  PREFIX template hipError_t xr2c_w<float, W>(int, bool, const XArgs<float>&, hipStream_t);                   \
  PREFIX template hipError_t xc2r_w<double, W>(int, bool, const XArgs<double>&, hipStream_t);                 \
  PREFIX template hipError_t xc2r_w<float, W>(int, bool, const XArgs<float>&, hipStream_t);                   \
  PREFIX template hipError_t zfft_w<double, W>(bool, bool, const ZfArgs<double>&, int, hipStream_t);          \
  PREFIX template hipError_t zfft_w<float, W>(bool, bool, const ZfArgs<float>&, int, hipStream_t);            \
  PREFIX template hipError_t batch_xr2c_w<double, W>(int, bool, const BatchGrid<double>*, const long*, long,  \
                                                     const BatchPtrs&, const BatchLaunch&, hipStream_t);      \
  PREFIX template hipError_t batch_xr2c_w<float, W>(int, bool, const BatchGrid<float>*, const long*, long,    \
                                                    const BatchPtrs&, const BatchLaunch&, hipStream_t);       \
  PREFIX template hipError_t batch_xc2r_w<double, W>(int, bool, const BatchGrid<double>*, const long*, long,  \
                                                     const BatchPtrs&, const BatchLaunch&, hipStream_t);      \
  PREFIX template hipError_t batch_xc2r_w<float, W>(int, bool, const BatchGrid<float>*, const long*, long,    \
                                                    const BatchPtrs&, const BatchLaunch&, hipStream_t);       \
  PREFIX template hipError_t batch_zfft_w<double, W>(bool, bool, const BatchGrid<double>*, const long*, long, \
                                                     const BatchLaunch&, hipStream_t);                        \
  PREFIX template hipError_t batch_zfft_w<float, W>(bool, bool, const BatchGrid<float>*, const long*, long,   \
                                                    const BatchLaunch&, hipStream_t);

}  // namespace ibp

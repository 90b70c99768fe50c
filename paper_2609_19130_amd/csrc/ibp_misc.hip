// Discrete divergence of a staggered velocity field: the right-hand side of
// the elliptic problem is (div u* - q) / (alpha dt) (paper, eq. ``elliptic``).
// u[j][k][i] sits on the x face at x = i dx, w[j][k][i] on the z face at
// z = k dz (both periodic), v[j][k][i] on the y face yf[j] (ny+1 rows).
#include <algorithm>

#include "ibp_internal.hpp"

namespace ibp {

// Both kernels march along y: a block owns a tile of KR consecutive z rows
// (all nx columns) and walks NJ consecutive y planes of it, keeping the
// values it needs from the planes below and above in registers, so every
// field is read from memory once (plus one z halo row per tile and one y
// halo plane per walk).  Tiles of a plane follow each other in block order,
// so the z neighbours of a tile's edge rows are read by blocks running at
// the same time.  NT threads own TILE / NT cells each: cell c of the tile
// (c = t + NT m) is row c / nx, column c % nx.  Two shapes: 512 threads over
// 2048-cell tiles (nx <= 2048; the faster of the shapes measured), and 512
// threads over 4096-cell tiles for wider rows (1024-thread blocks would cap
// the registers at 128 and spill).
constexpr int kMarchThreads = 512, kMarchTile = 2048;
constexpr int kMarchThreadsWide = 512, kMarchTileWide = 4096;
// LDS of the projection: (kr + 2) rows of nx, at most three times the tile
constexpr int kProjLds = 3 * kMarchTile, kProjLdsWide = 3 * kMarchTileWide;
// blocks per launch to aim for, and the longest walk along y
constexpr int kMarchBlocks = 1024, kMarchMaxPlanes = 32;

struct MarchShape {
  int kr;     // z rows per tile
  int ntk;    // tiles per plane
  int nj;     // y planes per block
  int nbj;    // blocks along y
};

// Blocks of a launch go to the XCDs in turn (block b to XCD b mod 8), and
// each XCD has its own L2.  The march kernels renumber blocks so that every
// XCD takes a contiguous range of tiles: neighbouring tiles of one plane,
// which read each other's edge rows, then share an L2.  Only the speed
// depends on the dispatch order; any order computes the same result.
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_block(int b, int nb) {
  const int q = nb / kXcds, r = nb % kXcds;
  const int x = b % kXcds, i = b / kXcds;
  return x < r ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

inline MarchShape march_shape(int nx, int ny, int nz, int tile, int max_planes = kMarchMaxPlanes) {
  MarchShape m;
  m.kr = std::max(1, std::min(nz, tile / nx));
  m.ntk = (nz + m.kr - 1) / m.kr;
  // enough blocks to fill the device with at least 4 planes each
  m.nj = std::max(4, std::min(max_planes, (int)((long)ny * m.ntk / kMarchBlocks)));
  m.nj = std::min(m.nj, ny);
  m.nbj = (ny + m.nj - 1) / m.nj;
  return m;
}

// Discrete divergence: v(j + 1) of a plane is v(j) of the next one; the
// x and z neighbours u(i + 1), w(k + 1) come from the same or the next row
// (cache hits, apart from each tile's last row).
template <int NT, int TILE>
__global__ __launch_bounds__(NT) void k_divergence(DivArgs A, MarchShape S) {
  constexpr int kMarchCells = TILE / NT;
  const int blk = xcd_block(blockIdx.x, gridDim.x);
  const int tk = blk % S.ntk, bj = blk / S.ntk;
  const int j0 = bj * S.nj, j1 = min(A.ny, j0 + S.nj);
  const int k0 = tk * S.kr, nx = A.nx;
  const long plane = (long)nx * A.nz;
  const int ncell = min(S.kr, A.nz - k0) * nx;
  int off[kMarchCells], offu[kMarchCells], offw[kMarchCells];   // within a plane (< 2^24)
  bool live[kMarchCells];
  double vb[kMarchCells];
#pragma unroll
  for (int m = 0; m < kMarchCells; ++m) {
    const int c = threadIdx.x + NT * m;
    live[m] = c < ncell;
    const int kk = live[m] ? c / nx : 0, i = live[m] ? c - kk * nx : 0;
    const int k = k0 + kk;
    off[m] = k * nx + i;
    offu[m] = k * nx + (i + 1 == nx ? 0 : i + 1);
    offw[m] = (k + 1 == A.nz ? 0 : k + 1) * nx + i;
    vb[m] = live[m] ? A.v[(long)j0 * plane + off[m]] : 0.0;
  }
  for (int j = j0; j < j1; ++j) {
    const long pj = (long)j * plane;
    const double* u = A.u + pj;
    const double* w = A.w + pj;
    const double* vt_row = A.v + pj + plane;
    const double* q = A.q ? A.q + pj : nullptr;
    double* f = A.f + pj;
    const double rdyf = A.dyf[j];
#pragma unroll
    for (int m = 0; m < kMarchCells; ++m) {
      if (!live[m]) continue;
      const double vt = vt_row[off[m]];
      const double du = u[offu[m]] - u[off[m]];
      const double dw = w[offw[m]] - w[off[m]];
      const double dv = vt - vb[m];
      double d = du * A.idx + dv / rdyf + dw * A.idz;
      if (q) d -= q[off[m]];
      f[off[m]] = d * A.scale;
      vb[m] = vt;
    }
  }
}

// Projection of the provisional velocity and pressure update, one pass over
// the cells (paper, eqs. ``velsolen`` and ``pressure``):
//   u -= adt (phi[i] - phi[i-1]) / dx,   w -= adt (phi[k] - phi[k-1]) / dz,
//   v on face j (1 <= j < ny) -= adt (phi[j] - phi[j-1]) / dyc_j,
//   p += phi - visc L_h phi.
// Wall faces of v: unchanged at a Neumann wall; at a Dirichlet wall (phi = 0
// on the face) the one-sided gradient over the half cell.  Cell (j,k,i)
// updates the faces west, south and below it (plus the upper wall face when
// j = ny-1), so every face has one writer.  The phi tile of the current
// plane, with one halo row on each z side, sits in LDS for the x and z
// neighbours; phi of the planes below and above, at the thread's own cells,
// in registers.
// LDS: capacity in doubles, at least (kr + 2) nx.
template <int NT, int TILE, int LDS>
__global__ __launch_bounds__(NT) void k_project(ProjArgs A, MarchShape S) {
  constexpr int kMarchCells = TILE / NT;
  __shared__ double tile[LDS];   // (kr + 2) rows of nx: z rows k0 - 1 .. k0 + kr
  const int blk = xcd_block(blockIdx.x, gridDim.x);
  const int tk = blk % S.ntk, bj = blk / S.ntk;
  const int j0 = bj * S.nj, j1 = min(A.ny, j0 + S.nj);
  const int k0 = tk * S.kr, nx = A.nx, nz = A.nz;
  const int kr = min(S.kr, nz - k0);
  const long plane = (long)nx * nz;
  const int ncell = kr * nx;
  int tc[kMarchCells], txm[kMarchCells], txp[kMarchCells];   // tile index of the cell and its x neighbours
  int off[kMarchCells];                                      // within a plane (< 2^24)
  bool live[kMarchCells];
#pragma unroll
  for (int m = 0; m < kMarchCells; ++m) {
    const int c = threadIdx.x + NT * m;
    live[m] = c < ncell;
    const int kk = live[m] ? c / nx : 0, i = live[m] ? c - kk * nx : 0;
    off[m] = (k0 + kk) * nx + i;
    tc[m] = (kk + 1) * nx + i;
    txm[m] = (kk + 1) * nx + (i == 0 ? nx - 1 : i - 1);
    txp[m] = (kk + 1) * nx + (i + 1 == nx ? 0 : i + 1);
  }
  // Tile row r holds z row (k0 - 1 + r) mod nz.  Each thread writes its own
  // cells (rows 1..kr) from registers; the two halo rows come from memory.
  auto fill = [&](int j, const double* own) {
#pragma unroll
    for (int m = 0; m < kMarchCells; ++m)
      if (live[m]) tile[tc[m]] = own[m];
    const double* src = A.phi + (long)j * plane;
    const int klo = k0 == 0 ? nz - 1 : k0 - 1, khi = k0 + kr == nz ? 0 : k0 + kr;
    for (int e = threadIdx.x; e < 2 * nx; e += NT) {
      const int hi = e >= nx, i = e - hi * nx;
      tile[hi ? (kr + 1) * nx + i : i] = src[(hi ? khi : klo) * nx + i];
    }
  };
  double pm[kMarchCells], pc[kMarchCells], pp[kMarchCells];
#pragma unroll
  for (int m = 0; m < kMarchCells; ++m) {
    pm[m] = (live[m] && j0 > 0) ? A.phi[(long)(j0 - 1) * plane + off[m]] : 0.0;   // wall value 0 beyond a wall
    pc[m] = live[m] ? A.phi[(long)j0 * plane + off[m]] : 0.0;
  }
  fill(j0, pc);
  const double ax = A.adt * A.idx, az = A.adt * A.idz;
  const double cxx = A.idx * A.idx, czz = A.idz * A.idz;
  for (int j = j0; j < j1; ++j) {
    const long pj = (long)j * plane;
    const double* phin = A.phi + pj + plane;
    double* u = A.u + pj;
    double* v = A.v + pj;
    double* w = A.w + pj;
    double* p = A.p ? A.p + pj : nullptr;
    const bool wall_hi = j + 1 == A.ny && A.dir_hi;
    // every global load of the plane is issued before the barrier
    double uo[kMarchCells], vo[kMarchCells], wo[kMarchCells], po[kMarchCells], vh[kMarchCells];
#pragma unroll
    for (int m = 0; m < kMarchCells; ++m) {
      pp[m] = (live[m] && j + 1 < A.ny) ? phin[off[m]] : 0.0;
      uo[m] = live[m] ? u[off[m]] : 0.0;
      wo[m] = live[m] ? w[off[m]] : 0.0;
      vo[m] = live[m] ? v[off[m]] : 0.0;
      po[m] = (live[m] && p) ? p[off[m]] : 0.0;
      vh[m] = (live[m] && wall_hi) ? v[off[m] + plane] : 0.0;
    }
    const double gy = j > 0 ? A.adt / A.dyc[j] : (A.dir_lo ? A.adt / (0.5 * A.dyf[0]) : 0.0);
    const double gyh = wall_hi ? A.adt / (0.5 * A.dyf[j]) : 0.0;
    const double ya = A.ya[j], yc = A.yc[j];
    __syncthreads();   // the tile of plane j is complete
#pragma unroll
    for (int m = 0; m < kMarchCells; ++m) {
      if (!live[m]) continue;
      const int o = off[m];
      const double c0 = pc[m];
      const double xm = tile[txm[m]], xp = tile[txp[m]];
      const double zm = tile[tc[m] - nx], zp = tile[tc[m] + nx];
      const double ym = pm[m], yp = pp[m];
      u[o] = uo[m] - ax * (c0 - xm);
      w[o] = wo[m] - az * (c0 - zm);
      if (j > 0 || A.dir_lo) v[o] = vo[m] - gy * (c0 - ym);   // ym = 0 on a Dirichlet wall face
      if (wall_hi) v[o + plane] = vh[m] - gyh * (0.0 - c0);
      if (p) {
        const double lap = (xp - 2.0 * c0 + xm) * cxx + (zp - 2.0 * c0 + zm) * czz + ya * (ym - c0) + yc * (yp - c0);
        p[o] = po[m] + (c0 - A.visc * lap);
      }
    }
    __syncthreads();   // every read of the tile is done
#pragma unroll
    for (int m = 0; m < kMarchCells; ++m) {
      pm[m] = pc[m];
      pc[m] = pp[m];
    }
    if (j + 1 < j1) fill(j + 1, pc);
  }
}

// Residual of an iterate without a transform (the mixed forms' convergence
// probe and final check): r = (f - m) - L_h phi at every cell, with the same
// 7-point operator and operation order as the residual x passes, reduced to
// the block's norm partials (one record per block, in block order).  phi
// marches along y as in the projection: the plane's tile with its z halo
// rows in LDS, the planes below and above in registers; f is read once.
template <int NT, int TILE, int LDS>
__global__ __launch_bounds__(NT) void k_resid_march(XArgs<float> A, MarchShape S) {
  constexpr int kMarchCells = TILE / NT;
  constexpr int kHalo = (2 * TILE + NT - 1) / NT;   // halo values per thread (2 rows of nx <= TILE)
  __shared__ double tile[LDS];   // (kr + 2) rows of nx: z rows k0 - 1 .. k0 + kr
  __shared__ double sh[kPartStride * (NT / kWave)];
  if (__builtin_amdgcn_readfirstlane(A.ctl->done)) return;
  if (A.probe && !__builtin_amdgcn_readfirstlane(A.ctl->probe)) return;
  const int blk = xcd_block(blockIdx.x, gridDim.x);
  const int tk = blk % S.ntk, bj = blk / S.ntk;
  const int j0 = bj * S.nj, j1 = min(A.ny, j0 + S.nj);
  const int k0 = tk * S.kr, nx = A.nx, nz = A.nz;
  const int kr = min(S.kr, nz - k0);
  const long plane = (long)nx * nz;
  const int ncell = kr * nx;
  const int klo = k0 == 0 ? nz - 1 : k0 - 1, khi = k0 + kr == nz ? 0 : k0 + kr;
  int tc[kMarchCells], txm[kMarchCells], txp[kMarchCells];
  int off[kMarchCells];
  bool live[kMarchCells];
#pragma unroll
  for (int m = 0; m < kMarchCells; ++m) {
    const int c = threadIdx.x + NT * m;
    live[m] = c < ncell;
    const int kk = live[m] ? c / nx : 0, i = live[m] ? c - kk * nx : 0;
    off[m] = (k0 + kk) * nx + i;
    tc[m] = (kk + 1) * nx + i;
    txm[m] = (kk + 1) * nx + (i == 0 ? nx - 1 : i - 1);
    txp[m] = (kk + 1) * nx + (i + 1 == nx ? 0 : i + 1);
  }
  // halo element e = threadIdx.x + NT q of the two z halo rows: its tile
  // slot and its offset within a plane
  int hslot[kHalo], hoff[kHalo];
#pragma unroll
  for (int q = 0; q < kHalo; ++q) {
    const int e = threadIdx.x + NT * q;
    const bool ok = e < 2 * nx;
    const int hi = e >= nx, i = ok ? e - hi * nx : 0;
    hslot[q] = ok ? (hi ? (kr + 1) * nx + i : i) : -1;
    hoff[q] = (hi ? khi : klo) * nx + i;
  }
  // Software pipeline: while plane j is reduced, the loads of plane j + 1
  // (f, the halo rows of phi) and of phi at plane j + 2 are in flight.
  double pm[kMarchCells], pc[kMarchCells], pp[kMarchCells], fo[kMarchCells], hv[kHalo];
#pragma unroll
  for (int m = 0; m < kMarchCells; ++m) {
    pm[m] = (live[m] && j0 > 0) ? A.phi[(long)(j0 - 1) * plane + off[m]] : 0.0;
    pc[m] = live[m] ? A.phi[(long)j0 * plane + off[m]] : 0.0;
    pp[m] = (live[m] && j0 + 1 < A.ny) ? A.phi[(long)(j0 + 1) * plane + off[m]] : 0.0;
    fo[m] = live[m] ? A.f[(long)j0 * plane + off[m]] : 0.0;
  }
#pragma unroll
  for (int q = 0; q < kHalo; ++q) hv[q] = hslot[q] >= 0 ? A.phi[(long)j0 * plane + hoff[q]] : 0.0;
  NormAcc acc;
  const double mean = A.ctl->removed_mean;
  for (int j = j0; j < j1; ++j) {
    // the tile of plane j: own cells from registers, halo rows as loaded
#pragma unroll
    for (int m = 0; m < kMarchCells; ++m)
      if (live[m]) tile[tc[m]] = pc[m];
#pragma unroll
    for (int q = 0; q < kHalo; ++q)
      if (hslot[q] >= 0) tile[hslot[q]] = hv[q];
    // loads for the next plane
    const bool more = j + 1 < j1;
    double fn[kMarchCells], pn[kMarchCells];
#pragma unroll
    for (int m = 0; m < kMarchCells; ++m) {
      fn[m] = (live[m] && more) ? A.f[(long)(j + 1) * plane + off[m]] : 0.0;
      pn[m] = (live[m] && more && j + 2 < A.ny) ? A.phi[(long)(j + 2) * plane + off[m]] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < kHalo; ++q)
      hv[q] = (hslot[q] >= 0 && more) ? A.phi[(long)(j + 1) * plane + hoff[q]] : 0.0;
    const double dyfj = A.dyf[j], ya = A.ya[j], yc = A.yc[j];
    __syncthreads();   // the tile of plane j is complete
#pragma unroll
    for (int m = 0; m < kMarchCells; ++m) {
      if (!live[m]) continue;
      const double c0 = pc[m];
      const double xm = tile[txm[m]], xp = tile[txp[m]];
      const double zm = tile[tc[m] - nx], zp = tile[tc[m] + nx];
      const double L0 = (xp - 2.0 * c0 + xm) * A.idx2 + (zp + zm - 2.0 * c0) * A.idz2 + ya * (pm[m] - c0) +
                        yc * (pp[m] - c0);
      const double f0 = fo[m] - mean;
      acc.one(f0 - L0, f0, dyfj * dyfj);
      acc.phi_one(c0, dyfj);
    }
    __syncthreads();   // every read of the tile is done
#pragma unroll
    for (int m = 0; m < kMarchCells; ++m) {
      pm[m] = pc[m];
      pc[m] = pp[m];
      pp[m] = pn[m];
      fo[m] = fn[m];
    }
  }
  acc.write<NT, true>(A.part, blockIdx.x, sh);
}

// The residual-only pass's blocks (= its partial records), 0 when the
// marching kernel does not take the grid.
constexpr int kResidMaxPlanes = 32;
long resid_march_blocks(int nx, int ny, int nz) {
  if (nx > kMarchTileWide || (long)nx * nz >= (1L << 30)) return 0;
  const MarchShape S = march_shape(nx, ny, nz, nx <= kMarchTile ? kMarchTile : kMarchTileWide, kResidMaxPlanes);
  return (long)S.ntk * S.nbj;
}

hipError_t launch_resid_march(const XArgs<float>& a, hipStream_t s) {
  if (a.nx > kMarchTileWide || (long)a.nx * a.nz >= (1L << 30)) return hipErrorInvalidValue;
  if (a.nx <= kMarchTile) {
    const MarchShape S = march_shape(a.nx, a.ny, a.nz, kMarchTile, kResidMaxPlanes);
    hipLaunchKernelGGL((k_resid_march<kMarchThreads, kMarchTile, kProjLds>), dim3((unsigned)(S.ntk * S.nbj)),
                       dim3(kMarchThreads), 0, s, a, S);
  } else {
    const MarchShape S = march_shape(a.nx, a.ny, a.nz, kMarchTileWide, kResidMaxPlanes);
    hipLaunchKernelGGL((k_resid_march<kMarchThreadsWide, kMarchTileWide, kProjLdsWide>),
                       dim3((unsigned)(S.ntk * S.nbj)), dim3(kMarchThreadsWide), 0, s, a, S);
  }
  return hipGetLastError();
}

hipError_t launch_project(const ProjArgs& a, hipStream_t s) {
  if (a.nx > kMarchTileWide || (long)a.nx * a.nz >= (1L << 30)) return hipErrorInvalidValue;
  if (a.nx <= kMarchTile) {
    const MarchShape S = march_shape(a.nx, a.ny, a.nz, kMarchTile);
    hipLaunchKernelGGL((k_project<kMarchThreads, kMarchTile, kProjLds>), dim3((unsigned)(S.ntk * S.nbj)),
                       dim3(kMarchThreads), 0, s, a, S);
  } else {
    const MarchShape S = march_shape(a.nx, a.ny, a.nz, kMarchTileWide);
    hipLaunchKernelGGL((k_project<kMarchThreadsWide, kMarchTileWide, kProjLdsWide>), dim3((unsigned)(S.ntk * S.nbj)),
                       dim3(kMarchThreadsWide), 0, s, a, S);
  }
  return hipGetLastError();
}

hipError_t launch_divergence(const DivArgs& a, hipStream_t s) {
  if (a.nx > kMarchTileWide || (long)a.nx * a.nz >= (1L << 30)) return hipErrorInvalidValue;
  if (a.nx <= kMarchTile) {
    const MarchShape S = march_shape(a.nx, a.ny, a.nz, kMarchTile);
    hipLaunchKernelGGL((k_divergence<kMarchThreads, kMarchTile>), dim3((unsigned)(S.ntk * S.nbj)),
                       dim3(kMarchThreads), 0, s, a, S);
  } else {
    const MarchShape S = march_shape(a.nx, a.ny, a.nz, kMarchTileWide);
    hipLaunchKernelGGL((k_divergence<kMarchThreadsWide, kMarchTileWide>), dim3((unsigned)(S.ntk * S.nbj)),
                       dim3(kMarchThreadsWide), 0, s, a, S);
  }
  return hipGetLastError();
}

}  // namespace ibp

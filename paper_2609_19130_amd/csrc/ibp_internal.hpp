// Internal declarations shared by the kernel translation units and the host
// side of libibpoisson.  Not part of the public C ABI (include/ibpoisson.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

#include "ibp_device.hpp"

namespace ibp {

// Spectrum layout: each kz row of a y plane starts on a 128-byte boundary
// (row stride rs = hp rounded up to 128 bytes) and each plane is padded by a
// further 128 bytes (plane stride ps = nz*rs + 128 bytes), which keeps the
// strided z-pass and line-solve accesses off a few HBM channels.
template <typename T>
inline long spec_row_stride(int hp) {
  const long e = 128 / (2 * (long)sizeof(T));
  return (hp + e - 1) / e * e;
}
template <typename T>
inline long spec_plane_stride(int hp, int nz) {
  return (long)nz * spec_row_stride<T>(hp) + 128 / (2 * (long)sizeof(T));
}

// Solve state kept in device memory.  The iteration-0 (0,0)-mode block
// re-initialises it at the start of every solve, before any kernel reads it,
// so no memset is ever enqueued (solves stay graph-capturable).
constexpr int kHistMax = 16;   // refinement residuals kept per solve
struct alignas(64) Ctl {
  int done;           // refinement finished: later kernels of the solve return at once
  int iters;          // refinement corrections applied after the initial solve
  int converged;      // 1: rel_residual <= rtol; 2: stopped at the FP64 floor (backward error); 0: not
  int nonfinite;      // non-finite value met in the right-hand side (or residual)
  double scale[2];    // FP32 input scale of refinement pass k is scale[k & 1]
  double fnorm2;      // ||f - m||_2^2
  double rnorm2;      // ||r||_2^2 of the latest residual
  double rmax;        // max |r| of the latest residual
  double removed_mean;
  double rel_residual;
  double phimean;     // volume-weighted mean of the iterate read by the latest residual pass
  double rel_residual_vw;   // ||V r||_2 / ||V (f - m)||_2, V the cell volumes
  double backward_error;    // ||r||_inf / (||L_h||_inf ||phi||_inf + ||f - m||_inf)
  int nhist;                // entries of hist
  int probe;                // 1: the next pass first tests the iterate with a residual-only pass
  double hist[kHistMax];    // rel_residual of the iterate after k corrections, k = 0, 1, ...
};

// Normwise backward error at which the refinement stops although rtol is
// not reached: the iterate is then as accurate as its FP64 representation
// allows (FP64 direct solutions measure 1.5-2.5 unit roundoffs on the
// benchmark grids), and further corrections cannot lower the residual.
constexpr double kEtaFloor = 8.0 * 1.1102230246251565e-16;

// x R2C input: f itself (PLAIN), the FP64 residual of the current iterate
// (RESID; RESID_ONLY reduces it without transforming), or f assembled on the
// fly from the provisional velocity and mass sources (DIV).
enum XMode { XM_PLAIN = 0, XM_RESID = 1, XM_RESID_ONLY = 2, XM_DIV = 3 };
enum CMode { CM_SET = 0, CM_ADD = 1 };

// Per-block norm partials of an x pass; `in` is what the pass transforms (f,
// or the residual r = f - m - L_h phi in the residual modes) and `fm` the
// right-hand side with its mean removed (residual modes; f otherwise):
//   [0] sum in^2          [1] sum fm^2          [2] max |in|
//   [3] non-finite count  [4] sum_j dyf_j phi   [5] sum dyf_j^2 in^2
//   [6] sum dyf_j^2 fm^2  [7] max |phi|         [8] max |fm|
// Slots 4, 5, 6 and 7 are filled by the residual modes only.
constexpr int kPartStride = 9;
#define IBP_PART_IS_MAX {false, false, true, false, false, false, false, true, true}

struct NormAcc {
  double in2 = 0.0, f2 = 0.0, imax = 0.0, bad = 0.0, wphi = 0.0, win2 = 0.0, wf2 = 0.0, pmax = 0.0, fmx = 0.0;
  // one residual or right-hand-side pair (in0, in1) with its (f - m) pair; w2 = dyf_j^2
  __device__ __forceinline__ void pair(double in0, double in1, double fm0, double fm1, double w2) {
    in2 += in0 * in0 + in1 * in1;
    f2 += fm0 * fm0 + fm1 * fm1;
    imax = fmax(imax, fmax(fabs(in0), fabs(in1)));
    if (!isfinite(in0) || !isfinite(in1)) bad += 1.0;
    win2 += w2 * (in0 * in0 + in1 * in1);
    wf2 += w2 * (fm0 * fm0 + fm1 * fm1);
    fmx = fmax(fmx, fmax(fabs(fm0), fabs(fm1)));
  }
  // a right-hand-side pair of a non-residual pass (in = f): only the plain
  // norms (sum, max, non-finite count); write<NT, false> derives the rest
  __device__ __forceinline__ void rhs_pair(double in0, double in1) {
    in2 += in0 * in0 + in1 * in1;
    imax = fmax(imax, fmax(fabs(in0), fabs(in1)));
    if (!isfinite(in0) || !isfinite(in1)) bad += 1.0;
  }
  __device__ __forceinline__ void rhs_one(double in0) {
    in2 += in0 * in0;
    imax = fmax(imax, fabs(in0));
    if (!isfinite(in0)) bad += 1.0;
  }
  __device__ __forceinline__ void one(double in0, double fm0, double w2) {
    in2 += in0 * in0;
    f2 += fm0 * fm0;
    imax = fmax(imax, fabs(in0));
    if (!isfinite(in0)) bad += 1.0;
    win2 += w2 * (in0 * in0);
    wf2 += w2 * (fm0 * fm0);
    fmx = fmax(fmx, fabs(fm0));
  }
  // the iterate's values at the cells of a residual pair (dyf = dyf_j)
  __device__ __forceinline__ void phi_pair(double p0, double p1, double dyf) {
    wphi += dyf * (p0 + p1);
    pmax = fmax(pmax, fmax(fabs(p0), fabs(p1)));
  }
  __device__ __forceinline__ void phi_one(double p0, double dyf) {
    wphi += dyf * p0;
    pmax = fmax(pmax, fabs(p0));
  }
  // block-reduce and write the block's partials (thread 0); every thread
  // calls it.  RESID: all slots; otherwise only the right-hand side's
  // (fm = in, no phi, no weighted sums).
  template <int NT, bool RESID, typename Ptr>
  __device__ __forceinline__ void write(Ptr part, long blk, double* sh) {
    if constexpr (RESID) {
      double v[kPartStride] = {in2, f2, imax, bad, wphi, win2, wf2, pmax, fmx};
      const bool ism[kPartStride] = IBP_PART_IS_MAX;
      block_reduce<kPartStride, NT>(v, ism, sh);
      if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < kPartStride; ++q) part[blk * kPartStride + q] = v[q];
      }
    } else {
      double v[3] = {in2, imax, bad};
      const bool ism[3] = {false, true, false};
      block_reduce<3, NT>(v, ism, sh);
      if (threadIdx.x == 0) {
        const double w[kPartStride] = {v[0], v[0], v[1], v[2], 0.0, 0.0, 0.0, 0.0, v[1]};
#pragma unroll
        for (int q = 0; q < kPartStride; ++q) part[blk * kPartStride + q] = w[q];
      }
    }
  }
};

template <typename T>
struct XArgs {
  const double* f;       // right-hand side [ny][nz][nx]
  const double* phi;     // current iterate (residual modes)
  double* out;           // solution [ny][nz][nx] (C2R)
  Cx<T>* spec;           // half spectrum: (j, kz, kx) at j*ps + kz*rs + kx, kx < hp
  double* rowsum;        // [ny*nz] FP64 sums of each transformed row
  double* part;          // [nblocks][kPartStride]
  const double* phi00;   // [ny] (0,0)-mode solution (C2R)
  Ctl* ctl;
  const Cx<T>* twx;      // W_nx^e, e < nx
  const double* ya;      // FP64 face coefficients of the y operator (residual)
  const double* yc;
  const double* dyf;     // cell widths (volume weights of the mean of phi)
  FftPlan fp;            // length h = nx/2
  int nx, ny, nz, h, hp;
  long rs, ps;           // spectrum row and plane strides (elements)
  int rows_per_block;
  long row_begin;        // rows [row_begin, nrows) of the [ny][nz] row space; a multiple of rows_per_block
  long nrows;            // end row (ny * nz for a whole-grid pass)
  int parts;             // write the per-block norm partials
  double idx2, idz2;     // 1/dx^2, 1/dz^2
  double out_scale;      // 1/(h nz): normalisation of the two inverse transforms
  double inv_nxnz;
  int iter;              // refinement pass (selects ctl->scale slot)
  // XM_DIV: f = (D u - q) * rscale from u, w [ny][nz][nx] (x and z faces),
  // v [ny+1][nz][nx] (y faces) and q [ny][nz][nx] (may be null)
  const double* u;
  const double* v;
  const double* w;
  const double* q;
  double idx, idz, rscale;
  // Bluestein x transforms (fp.blu): LDS row stride hs (0: h) and the chirp,
  // filter and length-m twiddle tables
  int hs;
  const Cx<T>* bc;
  const Cx<T>* bb;
  const Cx<T>* bt;
  // XM_RESID_ONLY as a probe: runs only when the latest check predicted
  // convergence (ctl->probe)
  int probe = 0;
};

// f = (D u - q) * rscale for the two cells (2m, 2m+1) of row (j, k): the
// staggered divergence of the provisional velocity, minus the mass sources.
template <typename T>
__device__ __forceinline__ double2 assemble_pair(const XArgs<T>& A, long row, int j, int k, int m) {
  const int nx = A.nx, nz = A.nz;
  const long e = row * nx + 2 * m;
  const double2 uc = *reinterpret_cast<const double2*>(A.u + e);
  const double ur = A.u[row * nx + (2 * m + 2 == nx ? 0 : 2 * m + 2)];
  const double2 vb = *reinterpret_cast<const double2*>(A.v + e);
  const double2 vt = *reinterpret_cast<const double2*>(A.v + e + (long)nz * nx);
  const int kp = k + 1 == nz ? 0 : k + 1;
  const double2 wc = *reinterpret_cast<const double2*>(A.w + e);
  const double2 wn = *reinterpret_cast<const double2*>(A.w + ((long)j * nz + kp) * nx + 2 * m);
  const double dyf = A.dyf[j];   // same operation order as the divergence kernel
  double f0 = (uc.y - uc.x) * A.idx + (vt.x - vb.x) / dyf + (wn.x - wc.x) * A.idz;
  double f1 = (ur - uc.y) * A.idx + (vt.y - vb.y) / dyf + (wn.y - wc.y) * A.idz;
  if (A.q) {
    const double2 qq = *reinterpret_cast<const double2*>(A.q + e);
    f0 -= qq.x;
    f1 -= qq.y;
  }
  return make_double2(f0 * A.rscale, f1 * A.rscale);
}

// The same for the single cell m of a row of odd length nx.
template <typename T>
__device__ __forceinline__ double assemble_one(const XArgs<T>& A, long row, int j, int k, int m) {
  const int nx = A.nx, nz = A.nz;
  const long e = row * nx + m;
  const double uc = A.u[e];
  const double ur = A.u[row * nx + (m + 1 == nx ? 0 : m + 1)];
  const double vb = A.v[e];
  const double vt = A.v[e + (long)nz * nx];
  const int kp = k + 1 == nz ? 0 : k + 1;
  const double wc = A.w[e];
  const double wn = A.w[((long)j * nz + kp) * nx + m];
  const double dyf = A.dyf[j];   // same operation order as the divergence kernel
  double f0 = (ur - uc) * A.idx + (vt - vb) / dyf + (wn - wc) * A.idz;
  if (A.q) f0 -= A.q[e];
  return f0 * A.rscale;
}

template <typename T>
struct ZfArgs {
  Cx<T>* spec;
  const Cx<T>* twz;      // W_nz^e, e < nz
  Ctl* ctl;
  FftPlan fp;            // length nz
  int nz, hp, cols;      // cols: kx columns per block
  long rs, ps;           // spectrum row and plane strides (elements)
  int check_done;
  int plane0;            // first y plane of this launch
  // Bluestein z transforms (fp.blu): LDS column stride zss (0: nz + 1) and
  // the chirp, filter and length-m twiddle tables
  int zss;
  const Cx<T>* bc;
  const Cx<T>* bb;
  const Cx<T>* bt;
};

template <typename T, typename U>   // T: spectral storage, U: line-solve arithmetic
struct YArgs {
  Cx<T>* spec;
  const U* lamx;         // [hp]
  const U* lamz;         // [nz]
  const U* ya;           // [ny] face coefficients: sub- and super-diagonal of the y operator
  const U* yc;
  Ctl* ctl;
  long Q;                // nz * rs column slots (kx >= hp are padding)
  long rs, ps;           // spectrum row and plane strides (elements)
  int ny, hp, check_done;
  int singular;          // Neumann at both walls: column (0,0) is left to the FP64 (0,0) path
  // IBP_MIXED_F64INV: the solution goes to this FP64 half spectrum (row and
  // plane strides out_rs, out_ps) instead of back into `spec`; add_iter > 0:
  // added to it instead, divided by the input scale ctl->scale[add_iter & 1]
  Cx<double>* out64;
  long out_rs, out_ps;
  int add_iter = 0;
};

// IBP_MIXED_F64INV, first correction without the initial iterate: the FP64
// inverse z transform of the FP32 right-hand-side spectrum (strides irs,
// ips) into an FP64 half spectrum (ors, ops).  zero00: the (kx, kz) = (0, 0)
// coefficient is dropped (the singular problem's plane means come from the
// FP64 row sums instead).
struct ZupArgs {
  const Cx<float>* in;
  long irs, ips;
  Cx<double>* out;
  long ors, ops;
  const Cx<double>* twz;   // FP64 W_nz^e
  int nz, hp, ny;
  int zero00;
};
// ... and the x pass that follows it: per row, t = FP64 inverse x transform
// of the z-inverted spectrum (x.out_scale included), r0 = f - t - ghat[j] /
// (nx nz) (the plane mean only when zero00 was set), written as the FP32
// half spectrum of r0 * ctl->scale[x.iter & 1] (x.spec), with the FP64 row
// sums of r0 (x.rowsum) and its norm partials (x.part).
struct RtArgs {
  XArgs<float> x;
  const Cx<double>* t64;
  long trs, tps;
  const Cx<double>* twx64;   // FP64 W_nx^e
  const double* ghat;
  int sub_mean;
};
hipError_t launch_zinv_up(const ZupArgs& a, hipStream_t s);

// Register Bluestein transforms (ibp_bluereg.hip) for lengths n <= 1024 with
// a prime factor above 11; M: the convolution length (a power of two >=
// 2n - 1, <= 2048); tables in the args' bc (chirp), bb (filter transform)
// and bt (W_M).  z: forward or inverse over nplanes planes from a.plane0;
// x: whole rows of nx points, two per line (R2C: FP64 right-hand side pass;
// C2R: set or add).
template <typename T>
hipError_t launch_zblu_reg(bool inverse, const ZfArgs<T>& a, int M, int nplanes, hipStream_t s);
template <typename T>
hipError_t launch_xblu_r2c(const XArgs<T>& a, int M, hipStream_t s);
template <typename T>
hipError_t launch_xblu_c2r(int mode, const XArgs<T>& a, int M, hipStream_t s);
hipError_t launch_x_roundtrip(const RtArgs& a, hipStream_t s);

struct ZeroArgs {        // FP64 (0,0) mode and solve control
  const double* rowsum;
  double* ghat;          // [ny] plane sums
  int* ticket;           // completion counter of the (0,0)-mode blocks (0 between launches)
  double* phi00;
  const double* dyf;     // [ny]
  const double* dyc;     // [ny+1], entries 1..ny-1 used
  const double* part;
  long nparts;
  Ctl* ctl;
  int nx, ny, nz;
  int init;              // first (0,0) solve of a solve call: re-initialise ctl
  int mixed;
  int iter;
  int final_pass;
  double rtol;
  double dyf_sum;        // sum_j dyf_j
  int singular;          // Neumann at both walls: remove the mean, solve (0,0) by flux integration
  double lnorm;          // ||L_h||_inf (largest absolute row sum of the operator)
  int probe = 0;         // check of a probe pass: stops on convergence, else leaves the state to the next check
  int nostop = 0;        // check that records the residual and prepares the next correction but never stops
  int phi00_add = 0;     // (0,0) mode: add this solve's solution to phi00 instead of replacing it
  double* part2 = nullptr;   // [kCheckSplitMax][kPartStride]: first-level sums of the check's split reduction
};
// The convergence check reduces its partials in two launches once there are
// more than kCheckSplitMin of them: up to kCheckSplitMax blocks each sum a
// contiguous slice (in order), then one block reduces those sums.
constexpr long kCheckSplitMin = 2048;
constexpr int kCheckSplitMax = 256;

// Fused x/z pass (persistent).  The y planes are dealt out to one work
// queue per XCD (plane p to queue p % nq) and a block only serves the queue
// of the XCD it runs on, so a plane's producer and consumer blocks share
// one L2 and the intermediate half spectrum never needs a device-wide cache
// write-back or invalidation.  Round r of a queue holds the first-stage
// items of its r-th plane followed by the second-stage items of its
// (r - lag)-th plane; second-stage items of a plane wait until all its
// first-stage items are complete (per-plane counters in `done`).  Forward:
// x R2C then z FFT; inverse: z inverse FFT then x C2R.  The last block to
// finish checks that every queue was served and zeroes the counters.
constexpr int kMaxXcc = 16;
template <typename T>
struct FusedArgs {
  XArgs<T> x;
  ZfArgs<T> z;
  int* queue;            // [kMaxXcc]
  int* done;             // [ny]
  int* exit_count;
  int* error;            // 1: a dependency wait ran out, 2: a queue had no block (results invalid)
  int nfirst, nsecond;   // items per plane of the first and second stage
  int lag;
  int ny;
  int nq;                           // queues (XCDs)
  signed char xcc_queue[kMaxXcc];   // hardware XCC id -> queue (-1: none)
};

// ---------------------------------------------------------------- batches
// Many grids solved together: every stage is one launch whose blocks cover
// all grids.  Block b of a stage belongs to grid g with
// start[g] <= b < start[g + 1] (prefix offsets of the per-grid block counts)
// and runs that grid's block b - start[g].  Per-grid arguments live in a
// device table written once per batch; the right-hand side and solution
// pointers, which change from call to call, travel in the launch arguments.
constexpr int kBatchMax = 64;

template <typename T>
struct BatchGrid {
  XArgs<T> x;      // f, phi, out and iter are replaced at launch
  ZfArgs<T> z;     // check_done replaced at launch
  YArgs<T, T> y;   // check_done replaced at launch
  ZeroArgs zero;   // init, mixed, iter, final_pass replaced at launch
  int zcolblocks;  // z-pass column blocks per plane
  int yk;          // line-solve rows per lane for this grid (the batch's K, K/2 or K/4)
};

struct BatchPtrs {
  const double* f[kBatchMax];
  double* phi[kBatchMax];
};

struct BatchLaunch {
  int count;
  int iter;
  int init;
  int mixed;
  int final_pass;
  int check_done;
};

// ---------------------------------------------------------------- persistent batches
// One launch for the whole batched solve (ibp_persist.hip).  The items of a
// queue (one queue per XCD) are grouped in segments: the blocks of one stage
// of one grid, in queue order.  An item of a segment waits until counter
// `dep` reaches `need` (the grid's previous stage complete) and counts itself
// in counter `done`.
enum PersistKind {
  PK_XR2C = 0, PK_XRES = 1, PK_XRESONLY = 2, PK_XC2R = 3, PK_XC2R_ADD = 4,
  PK_ZF = 5, PK_ZI = 6, PK_Y0 = 7, PK_Y1 = 8, PK_Y2 = 9, PK_CHECK = 10
};
constexpr int PF_INIT = 1, PF_FINAL = 2, PF_CHECK_DONE = 4;   // segment flags

struct PersistSeg {
  long first;   // queue position of the segment's first item
  int g;        // grid
  int kind;     // PersistKind; PK_Y0/1/2: the line solve with K, K/2 or K/4 rows per lane
  int iter;     // refinement pass of the stage
  int flags;    // PF_*
  int done;     // counter the items increment
  int dep;      // counter the items wait on (-1: none)
  int need;     // value of `dep` that releases them
  int pad;
};

struct PersistArgs {
  const void* grids;        // BatchGrid<T>[count]
  const PersistSeg* seg;    // the queues' segments, queue q at [qseg[q], qseg[q + 1])
  const int* qseg;          // [nq + 1]
  const long* qitems;       // [nq] items per queue
  int* head;                // [kMaxXcc] claim counters (zero between launches)
  int* cnt;                 // [ncnt] completion counters (zero between launches)
  int* exit_count;          // (zero between launches)
  int ncnt;
  int nq;
  int mixed;
  int chunk;                // items a block claims at once
  signed char xcc_queue[kMaxXcc];   // hardware XCC id -> queue (-1: none)
  int* err[kBatchMax];      // per grid: 1 = a wait gave up, 2 = its queue had no block
};

// Lanes and rows per lane the persistent kernel is built for.
bool persist_shape_supported(int P, int K);
template <typename T>
hipError_t persist_blocks_per_cu(bool wide, int P, int K, int* per_cu);
template <typename T>
hipError_t launch_persist(bool wide, int P, int K, const PersistArgs& a, const BatchPtrs& p, int blocks,
                          hipStream_t s);

// Stages of a batched solve; each launcher covers every grid in one launch.
template <typename T>
hipError_t launch_batch_xr2c(int mode, bool small, bool wide, const BatchGrid<T>* d, const long* start, long nblocks, const BatchPtrs& p,
                             const BatchLaunch& l, hipStream_t s);
template <typename T>
hipError_t launch_batch_xc2r(int mode, bool small, bool wide, const BatchGrid<T>* d, const long* start, long nblocks, const BatchPtrs& p,
                             const BatchLaunch& l, hipStream_t s);
template <typename T>
hipError_t launch_batch_zfft(bool inverse, bool small, bool wide, const BatchGrid<T>* d, const long* start, long nblocks,
                             const BatchLaunch& l, hipStream_t s);
template <typename T>
hipError_t launch_batch_ytri(int P, int K, int M, const BatchGrid<T>* d, const long* start, long nblocks,
                             const BatchLaunch& l, hipStream_t s);
template <typename T>
hipError_t launch_batch_check(const BatchGrid<T>* d, const BatchLaunch& l, hipStream_t s);
// Columns per block of the batched line solve for lanes P, rows per lane K.
template <typename T>
int batch_ytri_cols(int P, int K, int want);
int batch_grid_rows_per_lane(int ny, int P, int K);
// Blocks that run the FP64 (0,0) mode at the start of a grid's line-solve launch.
constexpr int kZeroBlocks = 8;
__host__ __device__ inline int zero_blocks(int ny) { return ny < kZeroBlocks ? ny : kZeroBlocks; }

struct DivArgs {          // f = (D u - q) * scale; q may be null
  const double* u;
  const double* v;
  const double* w;
  const double* q;
  double* f;
  const double* dyf;
  int nx, ny, nz;
  double idx, idz, scale;
};

// Projection (u -= adt G phi) and pressure update (p += phi - visc L_h phi).
struct ProjArgs {
  const double* phi;
  double *u, *v, *w, *p;     // p may be null
  const double* dyf;         // [ny]
  const double* dyc;         // [ny+1], entries 1..ny-1
  const double* ya;          // face coefficients of L_h (wall rows carry the Dirichlet terms)
  const double* yc;
  int nx, ny, nz;
  int dir_lo, dir_hi;        // Dirichlet walls
  double idx, idz, adt, visc;
};
hipError_t launch_project(const ProjArgs& a, hipStream_t s);

// Factored viscous solve: apply one direction's precomputed line LU in place.
// `lu` holds four zero-padded tables of `npad` = P K entries (forward
// multipliers m, pivot reciprocals s, back-substitution multipliers t, the
// periodic Sherman-Morrison correction w), then the forward and backward
// lane-scan multipliers (log2 P steps of P entries each).
struct LineArgs {
  double* f;
  const double* lu;
  long npad;
  int n;                 // line length
  int cyclic;            // apply x -= w (x_0 + g x_{n-1})
  double g;
  long nouter;           // strided lines: outer count and stride
  long ostride;
  long ncol;             // strided: columns per outer index; contiguous: number of lines
  long stride;           // strided: element stride along a line
  int rev;               // 1: blocks in descending order (start on what the previous pass wrote last)
};
int line_shape(int n, int* P, int* K);   // lanes and rows per lane for lines of n (0: too long)
hipError_t launch_lines_contig(int P, int K, const LineArgs& a, hipStream_t s);
hipError_t launch_lines_strided(int P, int K, const LineArgs& a, hipStream_t s);
hipError_t launch_fill_zero(double* p, long n, hipStream_t s);

// ---------------------------------------------------------------- launchers
constexpr long kYTileBytes = 104 * 1024;          // staged line-solve tile per block (64 x 12 x 8 FP64: 99 KB)

template <typename T> int tile_x();
template <typename T> int tile_z();
template <> inline int tile_x<double>() { return kTileX64; }
template <> inline int tile_x<float>() { return kTileX32; }
template <> inline int tile_z<double>() { return kTileZ64; }
template <> inline int tile_z<float>() { return kTileZ32; }

// x passes cover rows [a.row_begin, a.nrows); z passes cover planes
// [a.plane0, a.plane0 + nplanes).
template <typename T>
hipError_t launch_xr2c(int mode, bool small, bool wide, const XArgs<T>& a, hipStream_t s);
template <typename T>
hipError_t launch_xc2r(int mode, bool small, bool wide, const XArgs<T>& a, hipStream_t s);
template <typename T>
hipError_t launch_zfft(bool inverse, bool small, bool wide, const ZfArgs<T>& a, int nplanes, hipStream_t s);
// M columns per block: `want` (2, 4, 8 or 16) if given, else 128-byte rows;
// capped by the LDS budget.
template <typename T, typename U>
hipError_t launch_ytri(int P, int K, int want, const YArgs<T, U>& a, const ZeroArgs& z, hipStream_t s);
// FP32 half spectrum in, FP64 arithmetic, FP64 half spectrum a.out64 out.
hipError_t launch_ytri_out64(int P, int K, const YArgs<float, double>& a, const ZeroArgs& z, hipStream_t s);
hipError_t launch_check(const ZeroArgs& z, hipStream_t s);
// The (0,0)-mode work of a line-solve pass on its own (zero_blocks(ny) blocks).
hipError_t launch_zero_mode(const ZeroArgs& z, hipStream_t s);

// Register-FFT kernels for power-of-two lengths 32..1024 (ibp_fastxz.hip).
template <typename T>
hipError_t launch_xr2c_fast(int mode, const XArgs<T>& a, hipStream_t s);
template <typename T>
hipError_t launch_xc2r_fast(int mode, const XArgs<T>& a, hipStream_t s);
template <typename T>
hipError_t launch_zfft_fast(bool inverse, const ZfArgs<T>& a, int nplanes, hipStream_t s);
long fast_x_rows_per_block(int h);

// Fused persistent forward (x R2C + z FFT) or inverse (z inverse + x C2R)
// pass; available when fused_supported(h, nz).  `blocks` persistent blocks.
constexpr int kFusedThreads = 512;
bool fused_supported(int h, int nz);
int fused_x_rows(int h);
int fused_z_cols(int nz);
template <typename T>
hipError_t launch_fused_fwd(const FusedArgs<T>& a, int blocks, hipStream_t s);
template <typename T>
hipError_t launch_fused_inv(int cmode, const FusedArgs<T>& a, int blocks, hipStream_t s);
// Resident blocks per compute unit of the fused kernels (minimum over the
// forward and inverse forms) for half length h.
template <typename T>
hipError_t fused_blocks_per_cu(int h, int* blocks);
// Hardware XCC id of `nblocks` blocks (one int each), for the XCD map.
hipError_t launch_xcc_probe(int* out, int nblocks, hipStream_t s);
template <typename T>
int fast_z_cols(int nz);
hipError_t launch_divergence(const DivArgs& a, hipStream_t s);
// Residual-only pass (norm partials of f - m - L_h phi, no transform) by the
// y-marching stencil kernel; resid_march_blocks: its partial records, 0 for
// grids it does not take (nx > 4096 or nx nz >= 2^30).
long resid_march_blocks(int nx, int ny, int nz);
hipError_t launch_resid_march(const XArgs<float>& a, hipStream_t s);


}  // namespace ibp

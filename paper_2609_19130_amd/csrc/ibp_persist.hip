// Persistent batched solve: every stage of every grid of a batch in one
// launch (paper: the batched 2-D FFTs of the "Fluid domain" parallelisation
// subsection, here extended to the whole solve of many uneven grids).
//
// Each grid is pinned to one XCD (accelerator complex die).  The host lays
// out, per XCD, a queue of work items: the blocks of every stage of the
// grids of that XCD, stage after stage per grid, the grids' stages
// interleaved along diagonals (stage s of the i-th grid next to stage s - 1
// of grid i + 1, ...) so that while one grid waits for a stage to finish the
// XCD runs stages of others.  A block serves the queue of the XCD it runs
// on: it claims the next item, waits until the stage that item depends on
// has completed (a per-grid, per-stage completion counter), runs the block
// body of the single-grid kernels, and counts the item done.
//
// Coherence: producer and consumer of a stage share the XCD's L2.  A
// producer's stores are in the L2 once its store counter drains; the
// consumer then invalidates its compute unit's L1 (an agent-scope acquire,
// which writes nothing back) before it reads.  No device-wide L2 write-back
// is needed between stages.  Claims are made in queue order and every
// dependency points to an earlier segment of the same queue, so the wait of
// a claimed item always ends; it is also bounded, raising the grid's error
// flag instead of hanging.
#include "ibp_internal.hpp"
#include "ibp_xz_kernels.hpp"
#include "ibp_ytri_body.hpp"

namespace ibp {

// Waves per SIMD the persistent kernel is compiled for: at 2 (up to 256
// VGPRs) no instance spills; at 3 every instance spills 120-530 bytes and
// the 64-grid batch still runs 5% (FP64) and 11% (mixed) faster.
#ifndef IBP_PERSIST_WAVES
#define IBP_PERSIST_WAVES 3
#endif

template <typename T, bool W, int P, int K0>
struct PersistShape {
  static constexpr int TLX = sizeof(T) == 8 ? kTileX64s : kTileX32s;
  static constexpr int TLZ = sizeof(T) == 8 ? kTileZ64s : kTileZ32s;
  static constexpr int M = kThreads / P;   // line-solve columns per block
  static constexpr long bx = (long)TLX * sizeof(Cx<T>);
  static constexpr long bz = (long)(TLZ + 64) * sizeof(Cx<T>);
  static constexpr long by = ytile_slots<M, P, K0>() * (long)sizeof(Cx<T>);
  static constexpr long buf = bx > bz ? (bx > by ? bx : by) : (bz > by ? bz : by);
};

// Segment of queue q holding queue position `item`: the last segment whose
// first item is <= item (wave-uniform binary search).
__device__ __forceinline__ int persist_segment(const PersistSeg* seg, int lo, int hi, long item) {
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (__builtin_amdgcn_readfirstlane((int)(seg[mid].first <= item))) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Item bodies: the single-grid block bodies on the grid's descriptor.
template <typename T, bool W, int MODE>
__device__ __forceinline__ void pb_x(const BatchGrid<T>* D, int g, const double* f, double* phi, int iter, long blk,
                                  Cx<T>* buf, double* sh) {
  using S = PersistShape<T, W, 32, 4>;
  XArgs<T> a = D[g].x;
  a.f = f;
  a.phi = phi;
  a.out = phi;
  a.iter = iter;
  if constexpr (MODE == XM_PLAIN || MODE == XM_RESID || MODE == XM_RESID_ONLY)
    xr2c_gen_body<T, MODE, S::TLX, W>(a, D[g].x.fp, blk, buf, sh);
  else
    xc2r_gen_body<T, MODE == 10 ? CM_SET : CM_ADD, S::TLX, W>(a, D[g].x.fp, blk, buf);
}

template <typename T, bool W, bool INV>
__device__ __forceinline__ void pb_z(const BatchGrid<T>* D, int g, int check_done, long blk, Cx<T>* buf) {
  using S = PersistShape<T, W, 32, 4>;
  ZfArgs<T> z = D[g].z;
  z.check_done = check_done;
  const int ncb = D[g].zcolblocks;
  zfft_gen_body<T, INV, S::TLZ, W>(z, D[g].z.fp, (int)(blk % ncb), blk / ncb, buf);
}

template <typename T, int M, int P, int K>
__device__ __forceinline__ void pb_y(const BatchGrid<T>* D, int g, int flags, int mixed, int iter, long blk,
                                  Cx<T>* buf) {
  YArgs<T, T> y = D[g].y;
  y.check_done = flags & PF_CHECK_DONE;
  ZeroArgs zr = D[g].zero;
  zr.init = (flags & PF_INIT) ? 1 : 0;
  zr.mixed = mixed;
  zr.iter = iter;
  zr.final_pass = 0;
  ytri_body<T, T, M, P, K>(y, zr, blk, buf);
}

template <typename T>
__device__ __forceinline__ void pb_check(const BatchGrid<T>* D, int g, int flags, int iter, double* sh) {
  ZeroArgs zr = D[g].zero;
  zr.init = 0;
  zr.mixed = 1;
  zr.iter = iter;
  zr.final_pass = (flags & PF_FINAL) ? 1 : 0;
  check_body<kThreads>(zr, sh);
}

template <typename T, bool W, int P, int K0>
__device__ __forceinline__ void persist_item(const PersistArgs& A, const BatchPtrs& Pt, const PersistSeg& sg,
                                             long blk, char* smem, double* sh) {
  using S = PersistShape<T, W, P, K0>;
  const BatchGrid<T>* D = static_cast<const BatchGrid<T>*>(A.grids);
  const int g = sg.g;
  Cx<T>* buf = reinterpret_cast<Cx<T>*>(smem);
  switch (sg.kind) {
    case PK_XR2C: pb_x<T, W, XM_PLAIN>(D, g, Pt.f[g], Pt.phi[g], sg.iter, blk, buf, sh); break;
    case PK_XC2R: pb_x<T, W, 10>(D, g, Pt.f[g], Pt.phi[g], sg.iter, blk, buf, sh); break;
    case PK_ZF: pb_z<T, W, false>(D, g, sg.flags & PF_CHECK_DONE, blk, buf); break;
    case PK_ZI: pb_z<T, W, true>(D, g, sg.flags & PF_CHECK_DONE, blk, buf); break;
    case PK_Y0: pb_y<T, S::M, P, K0>(D, g, sg.flags, A.mixed, sg.iter, blk, buf); break;
    case PK_Y1:
      if constexpr (K0 % 2 == 0) pb_y<T, S::M, P, K0 / 2>(D, g, sg.flags, A.mixed, sg.iter, blk, buf);
      break;
    case PK_Y2:
      if constexpr (K0 % 4 == 0) pb_y<T, S::M, P, K0 / 4>(D, g, sg.flags, A.mixed, sg.iter, blk, buf);
      break;
    default:
      if constexpr (sizeof(T) == 4) {   // refinement stages: FP32 spectra only
        if (sg.kind == PK_XRES)
          pb_x<T, W, XM_RESID>(D, g, Pt.f[g], Pt.phi[g], sg.iter, blk, buf, sh);
        else if (sg.kind == PK_XRESONLY)
          pb_x<T, W, XM_RESID_ONLY>(D, g, Pt.f[g], Pt.phi[g], sg.iter, blk, buf, sh);
        else if (sg.kind == PK_XC2R_ADD)
          pb_x<T, W, 11>(D, g, Pt.f[g], Pt.phi[g], sg.iter, blk, buf, sh);
        else if (sg.kind == PK_CHECK)
          pb_check<T>(D, g, sg.flags, sg.iter, sh);
      }
      break;
  }
}

template <typename T, bool W, int P, int K0>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(IBP_PERSIST_WAVES)))
void kp_batch(PersistArgs A, BatchPtrs Pt) {
  using S = PersistShape<T, W, P, K0>;
  __shared__ __attribute__((aligned(16))) char smem[S::buf];
  __shared__ double sh[(kThreads / kWave) * kPartStride];
  __shared__ int claimed;
  const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x) / kWave;
  const int lane = (int)threadIdx.x % kWave;
  const int q = __builtin_amdgcn_readfirstlane((int)A.xcc_queue[xcc_id()]);
  if (q >= 0) {
    const long total = A.qitems[q];
    const int s1 = A.qseg[q + 1] - 1;
    int si = A.qseg[q];    // current segment: a block's claims only move forward
    int verified = -1;     // segment whose dependency this block has seen met
    int pend_seg = -1, pend = 0;   // items done and not yet counted
    // count the pending items once every wave's stores have drained into the L2
    auto flush = [&]() {
      if (pend == 0) return;
      __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
      __syncthreads();
      if (wave == 0) atomicAdd(A.cnt + A.seg[pend_seg].done, lane == 0 ? pend : 0);
      pend = 0;
    };
    for (;;) {
      // claim A.chunk consecutive items (wave-uniform: all lanes of wave 0
      // take part, lane 0 adds): one claim and one completion count per chunk
      // (or per segment within it)
      if (wave == 0) {
        const int got = atomicAdd(A.head + q, lane == 0 ? A.chunk : 0);
        if (lane == 0) claimed = __builtin_amdgcn_readfirstlane(got);
      }
      __syncthreads();
      const long base = __builtin_amdgcn_readfirstlane((int)claimed);
      __syncthreads();
      if (base >= total) break;
      const long end = base + A.chunk < total ? base + A.chunk : total;
      for (long item = base; item < end; ++item) {
        si = persist_segment(A.seg, si, s1, item);
        const PersistSeg sg = A.seg[si];
        // never wait while holding uncounted items (they may be what is waited on)
        if (si != pend_seg) flush();
        if (sg.dep >= 0 && verified != si) {
          // a stage of one grid takes well under a millisecond; 2^17 polls
          // (~0.2 s) bound the wait
          if (wave == 0) wave_wait_count(A.cnt + sg.dep, sg.need, A.err[sg.g], 1 << 17);
          __syncthreads();
          // this compute unit's L1 may hold lines of an earlier stage: drop them
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
          verified = si;
        }
        persist_item<T, W, P, K0>(A, Pt, sg, item - sg.first, smem, sh);
        __syncthreads();   // the next item re-uses the LDS
        pend_seg = si;
        ++pend;
      }
      flush();
    }
    flush();
  }
  // the last block out checks that every queue was served and re-arms the
  // counters for the next launch
  if (wave == 0) {
    const int t = __builtin_amdgcn_readfirstlane(atomicAdd(A.exit_count, lane == 0 ? 1 : 0));
    if (t == (int)gridDim.x - 1) {
      for (int qq = 0; qq < A.nq; ++qq) {
        const int c = __builtin_amdgcn_readfirstlane(
            __hip_atomic_load(A.head + qq, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
        if (c < A.qitems[qq]) {   // a queue without a block: its grids were not solved
          for (int s = A.qseg[qq] + lane; s < A.qseg[qq + 1]; s += kWave)
            __hip_atomic_store(A.err[A.seg[s].g], 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
      }
      for (int i = lane; i < A.ncnt; i += kWave) A.cnt[i] = 0;
      if (lane < kMaxXcc) A.head[lane] = 0;
      if (lane == 0) *A.exit_count = 0;
    }
  }
}

template <typename T, bool W, int P, int K0>
static hipError_t persist_occ(int* per_cu) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(
      per_cu, reinterpret_cast<const void*>(&kp_batch<T, W, P, K0>), kThreads, 0);
}

// (lanes, rows per lane) shapes the persistent kernel is built for: the
// line-solve shapes of batches whose tallest grid has at most 512 rows
bool persist_shape_supported(int P, int K) {
  return (P == 32 && (K == 4 || K == 8 || K == 12)) || (P == 64 && K == 8);
}

template <typename T>
hipError_t persist_blocks_per_cu(bool wide, int P, int K, int* per_cu) {
  *per_cu = 0;
#define IBP_PERSIST_CASE(PP, KK)                                                          \
  if (P == PP && K == KK) return wide ? persist_occ<T, true, PP, KK>(per_cu) : persist_occ<T, false, PP, KK>(per_cu);
  IBP_PERSIST_CASE(32, 4)
  IBP_PERSIST_CASE(32, 8)
  IBP_PERSIST_CASE(32, 12)
  IBP_PERSIST_CASE(64, 8)
#undef IBP_PERSIST_CASE
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_persist(bool wide, int P, int K, const PersistArgs& a, const BatchPtrs& p, int blocks,
                          hipStream_t s) {
  auto go = [&](auto kern) {
    hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(kThreads), 0, s, a, p);
    return hipGetLastError();
  };
#define IBP_PERSIST_CASE(PP, KK) \
  if (P == PP && K == KK) return wide ? go(kp_batch<T, true, PP, KK>) : go(kp_batch<T, false, PP, KK>);
  IBP_PERSIST_CASE(32, 4)
  IBP_PERSIST_CASE(32, 8)
  IBP_PERSIST_CASE(32, 12)
  IBP_PERSIST_CASE(64, 8)
#undef IBP_PERSIST_CASE
  return hipErrorInvalidValue;
}

template hipError_t persist_blocks_per_cu<double>(bool, int, int, int*);
template hipError_t persist_blocks_per_cu<float>(bool, int, int, int*);
template hipError_t launch_persist<double>(bool, int, int, const PersistArgs&, const BatchPtrs&, int, hipStream_t);
template hipError_t launch_persist<float>(bool, int, int, const PersistArgs&, const BatchPtrs&, int, hipStream_t);

}  // namespace ibp

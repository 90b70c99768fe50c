// Host side of libibpoisson: argument validation, FP64 geometry and tables,
// workspace management and the enqueue order of the solve passes.  Every
// entry point is extern "C", returns a status and catches C++ exceptions.
#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/ibpoisson.h"
#include "ibp_host.hpp"
#include "ibp_internal.hpp"
#include "ibp_regfft.hpp"

using namespace ibp;

namespace {

constexpr int kVersion = 200;  // 0.2.0

inline size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

ibp_status_t from_hip(hipError_t e) {
  if (e == hipSuccess) return IBP_SUCCESS;
  if (e == hipErrorOutOfMemory) return IBP_ERROR_OUT_OF_MEMORY;
  return IBP_ERROR_HIP;
}

}  // namespace

struct ibp_plan_s {
  int nx = 0, ny = 0, nz = 0, h = 0, hp = 0;
  double Lx = 0, Lz = 0, dx = 0, dz = 0, dyf_sum = 0;
  int device = 0;
  ibp_precision_t prec = IBP_FP64;
  double rtol = 1e-10;
  int max_iters = 4;
  FftPlan fpx{}, fpz{};
  int yP = 32, yK = 2;   // line solve: lanes per column, rows per lane
  int ycols = 0;         // line-solve columns per block (0: 128-byte rows; set by the autotuner)
  int zc64max = 1, zc32max = 1;   // z-pass columns per block of the general kernel before tuning
  int zc64 = 1, zc32 = 1;   // z-pass kx columns per block
  int rb64 = 1, rb32 = 1;   // x-pass rows per block
  long nb64 = 1, nb32 = 1;  // x-pass blocks (transform passes)
  long nbro = 1;            // blocks of the residual-only pass
  bool xfast = false, zfast = false;   // register-FFT kernels for power-of-two lengths
  int xbm = 0, zbm = 0;   // register Bluestein convolution lengths of the x and z transforms (0: off)
  bool zsmall = false;                 // general z transform in the small tile
  bool xsmall = false;                 // general x transform in the small tile
  bool xwide = true, zwide = true;     // general transform needs the wide kernel family
  // fused persistent x/z passes (nz = nx and both lengths register-FFT sizes)
  bool fused = false;
  int fblocks64 = 0, fblocks32 = 0;   // persistent blocks (FP64 / FP32 spectrum)
  long nbf = 0;                       // x-row blocks of a fused pass (= its partials)
  // device tables
  void* tables = nullptr;
  const double *ya = nullptr, *yc = nullptr, *dyf = nullptr, *dyc = nullptr;
  const double *lamx = nullptr, *lamz = nullptr;
  const float *ya32 = nullptr, *yc32 = nullptr, *lamx32 = nullptr, *lamz32 = nullptr;
  const Cx<double>*twx = nullptr, *twz = nullptr;
  const Cx<float>*twx32 = nullptr, *twz32 = nullptr;
  // Bluestein tables (chirp, filter transform, length-m twiddles) of x and z
  const Cx<double>* bx64[3] = {nullptr, nullptr, nullptr};
  const Cx<double>* bz64[3] = {nullptr, nullptr, nullptr};
  const Cx<float>* bx32[3] = {nullptr, nullptr, nullptr};
  const Cx<float>* bz32[3] = {nullptr, nullptr, nullptr};
  // the x register Bluestein tables (whole rows of nx points), kept apart
  // from the general x kernels' (nx/2 or nx points, primes above 256)
  const Cx<double>* bxr64[3] = {nullptr, nullptr, nullptr};
  const Cx<float>* bxr32[3] = {nullptr, nullptr, nullptr};
  // workspace
  void* ws = nullptr;
  size_t ws_bytes = 0;
  bool ws_owned = false;
  Cx<double>* spec64 = nullptr;
  Cx<float>* spec32 = nullptr;
  double* rowsum = nullptr;
  double* phi00 = nullptr;
  double* ghat = nullptr;
  int* ticket = nullptr;
  int* fctl = nullptr;   // fused-pass counters: queues[16], exit count, error flag, pad[2], done[ny]
  int nq = 0;                               // XCD work queues of the fused passes
  signed char xcc_queue[kMaxXcc] = {0};     // hardware XCC id -> queue
  double* part = nullptr;
  Ctl* ctl = nullptr;
  const Ctl* info_ctl = nullptr;   // control block of the last solve
  hipStream_t last_stream = nullptr;
  bool solved = false;
  unsigned gen = 0;   // bumped when the precision, workspace or wall conditions change (batches check it)
  ibp_bc_t bc_lo = IBP_BC_NEUMANN, bc_hi = IBP_BC_NEUMANN;
  double lnorm = 0.0;   // ||L_h||_inf with the current wall conditions
  std::vector<double> ya_host, yc_host, dyf_host;   // Neumann face coefficients and cell widths
  std::vector<double> dyc_host;                      // centre distances, entries 1..ny-1
  // factored viscous solve (ibp_helmholtz_set): device factor tables per direction
  struct LineDir {
    int P = 0, K = 0, n = 0, cyclic = 0;
    long npad = 0, off = 0;   // table stride and offset in `helm` (doubles)
    double g = 0.0;
  };
  double* helm = nullptr;
  size_t helm_doubles = 0;
  bool helm_ready = false, helm_faces = false;
  ibp_bc_t helm_lo = IBP_BC_NEUMANN, helm_hi = IBP_BC_NEUMANN;
  LineDir hx, hz, hyc, hyf;
  bool singular() const { return bc_lo == IBP_BC_NEUMANN && bc_hi == IBP_BC_NEUMANN; }
  // chunked x/z passes: second stream and dependency events
  int chunk = 0;                   // y planes per chunk (0: whole grid per launch)
  hipStream_t s2 = nullptr;
  hipEvent_t ev_fork = nullptr;
  std::vector<hipEvent_t> ev_a, ev_b;
  // profiling: event pairs around launches, per pass id
  bool profiling = false;
  std::vector<hipEvent_t> ev_pool;
  std::vector<int> ev_pass;       // pass id of pair i (events 2i, 2i+1)
  size_t ev_used = 0;
};

namespace {

// fused-pass counter block: queues, exit count, error flag, padding, done[ny]
constexpr int kFctlQueue = 0, kFctlExit = kMaxXcc, kFctlError = kMaxXcc + 1, kFctlHead = kMaxXcc + 4;

// Largest absolute row sum of L_h: 4/dx^2 and 4/dz^2 from the periodic
// second differences (none for a single cell), 2 (a_j + c_j) from row j of
// the y operator (a, c are the face coefficients, wall terms included).
double operator_inf_norm(const ibp_plan_s* p, const std::vector<double>& a, const std::vector<double>& c) {
  double y = 0.0;
  for (int j = 0; j < p->ny; ++j) y = std::max(y, 2.0 * (a[j] + c[j]));
  const double x = p->nx > 1 ? 4.0 / (p->dx * p->dx) : 0.0;
  const double z = p->nz > 1 ? 4.0 / (p->dz * p->dz) : 0.0;
  return x + z + y;
}

// Norm partials: one per x-pass block; one per row bounds every x split and
// tile the tuner may choose.
long max_parts(const ibp_plan_s* p) {
  long nb = p->nb64 > p->nb32 ? p->nb64 : p->nb32;
  nb = nb > p->nbf ? nb : p->nbf;
  nb = nb > p->nbro ? nb : p->nbro;
  const long nrows = (long)p->ny * p->nz;
  return nb > nrows ? nb : nrows;
}

// Counters that kernels expect at zero between launches (each kernel that
// uses one re-arms it before it exits).
hipError_t reset_counters(ibp_plan_s* p) {
  hipError_t e = hipMemset(p->ticket, 0, sizeof(int));
  if (e == hipSuccess) e = hipMemset(p->fctl, 0, (size_t)(kFctlHead + p->ny) * sizeof(int));
  return e;
}

// Rows (x) or columns (z) per block of the general LDS transforms: whole
// tiles, or half tiles when the length has a prime factor above 11 (the
// direct-sum stage writes into the other half).
int x_tile_rows(const ibp_plan_s* p, int tile) {
  if (p->fpx.blu) return tile / p->fpx.m;
  return (p->fpx.any ? tile / 2 : tile) / p->h;
}
// Rows of this transform length fit the small x tile (FP64; FP32's is twice
// as large).  Lengths with a direct-sum stage keep the large tile: its work
// per block is the block's rows times h / 4 items, and one row of a half
// small tile leaves most threads idle (measured slower at h = 316 and 501).
bool x_small(const FftPlan& fpx, int h) { return !fpx.any && !fpx.blu && h <= kTileX64s; }
int x_tile64(const ibp_plan_s* p) { return p->xsmall ? kTileX64s : kTileX64; }
int x_tile32(const ibp_plan_s* p) { return p->xsmall ? kTileX32s : kTileX32; }
int z_tile_cols(const ibp_plan_s* p, int tile) {
  if (p->fpz.blu) return tile / (p->fpz.m + 1);
  return p->fpz.any ? (tile / 2) / (p->nz + 1) : tile / p->nz;
}
// A factorisation with a radix other than 2, 3, 4, 5, 8 (or Bluestein's
// convolution) needs the wide kernel family; the narrow one holds far fewer
// registers.
bool fft_wide(const FftPlan& fp) {
  if (fp.blu || fp.any) return true;
  for (int s = 0; s < fp.nst; ++s) {
    const int r = fp.radix[s];
    if (r != 2 && r != 3 && r != 4 && r != 5 && r != 8) return true;
  }
  return false;
}
// Lines of this length fit the small z tile (FP64; the FP32 one is twice as large).
bool z_small(const FftPlan& fpz, int nz) {
  if (fpz.blu) return false;
  return fpz.any ? nz + 1 <= kTileZ64s / 2 : nz <= kTileZ64s;
}

// The FP64 and FP32 half spectra are separate regions: the FP64 inverse
// passes of IBP_MIXED_F64INV read the FP32 one and write the FP64 one.
// x-pass rows per block and block counts for the plan's x tile (small or
// large LDS tile of the general kernels; the register kernels' rows are fixed).
void set_x_split(ibp_plan_s* p) {
  const long nrows = (long)p->ny * p->nz;
  p->nbro = (nrows + x_tile_rows(p, x_tile32(p)) - 1) / x_tile_rows(p, x_tile32(p));
  // the residual-only pass runs as the y-marching stencil kernel where it can
  if (const long nb = resid_march_blocks(p->nx, p->ny, p->nz)) p->nbro = nb;
  if (p->xfast) {
    p->rb64 = p->rb32 = (int)fast_x_rows_per_block(p->h);
  } else {
    p->rb64 = x_tile_rows(p, x_tile64(p));
    p->rb32 = x_tile_rows(p, x_tile32(p));
  }
  p->nb64 = (nrows + p->rb64 - 1) / p->rb64;
  p->nb32 = (nrows + p->rb32 - 1) / p->rb32;
}

// z-pass columns per block for the plan's z tile, divided by zdiv.
void set_z_split(ibp_plan_s* p, int zdiv) {
  p->zc64max = z_tile_cols(p, p->zsmall ? kTileZ64s : kTileZ64);
  p->zc32max = z_tile_cols(p, p->zsmall ? kTileZ32s : kTileZ32);
  p->zc64max = std::min(std::min(p->zc64max, 64), p->hp);
  p->zc32max = std::min(std::min(p->zc32max, 64), p->hp);
  p->zc64 = std::max(1, p->zc64max / zdiv);
  p->zc32 = std::max(1, p->zc32max / zdiv);
}

size_t spec64_bytes(const ibp_plan_s* p) {
  return (size_t)p->ny * spec_plane_stride<double>(p->hp, p->nz) * sizeof(Cx<double>);
}
size_t spec32_bytes(const ibp_plan_s* p) {
  return (size_t)p->ny * spec_plane_stride<float>(p->hp, p->nz) * sizeof(Cx<float>);
}

size_t workspace_bytes(const ibp_plan_s* p) {
  size_t b = align256(spec64_bytes(p)) + align256(2 * spec32_bytes(p));
  b += align256(2 * (size_t)p->ny * p->nz * sizeof(double));
  b += align256((size_t)p->ny * sizeof(double));   // phi00
  b += align256((size_t)p->ny * sizeof(double));   // ghat
  b += align256(sizeof(int));                      // ticket
  b += align256((size_t)(kFctlHead + p->ny) * sizeof(int)); // fused-pass counters
  b += align256((size_t)(2 * max_parts(p) + kCheckSplitMax) * kPartStride * sizeof(double));
  b += align256(sizeof(Ctl));
  return b;
}

void carve_workspace(ibp_plan_s* p) {
  char* c = static_cast<char*>(p->ws);
  p->spec64 = reinterpret_cast<Cx<double>*>(c);
  c += align256(spec64_bytes(p));
  p->spec32 = reinterpret_cast<Cx<float>*>(c);   // two FP32 half spectra (spec32_second)
  c += align256(2 * spec32_bytes(p));
  p->rowsum = reinterpret_cast<double*>(c);       // two row-sum arrays (rowsum_second)
  c += align256(2 * (size_t)p->ny * p->nz * sizeof(double));
  p->phi00 = reinterpret_cast<double*>(c);
  c += align256((size_t)p->ny * sizeof(double));
  p->ghat = reinterpret_cast<double*>(c);
  c += align256((size_t)p->ny * sizeof(double));
  p->ticket = reinterpret_cast<int*>(c);
  c += align256(sizeof(int));
  p->fctl = reinterpret_cast<int*>(c);
  c += align256((size_t)(kFctlHead + p->ny) * sizeof(int));
  p->part = reinterpret_cast<double*>(c);   // two partial regions (part_second), then the check's first-level sums
  c += align256((size_t)(2 * max_parts(p) + kCheckSplitMax) * kPartStride * sizeof(double));
  p->ctl = reinterpret_cast<Ctl*>(c);
}

// Register Bluestein for a transform of length n: lengths up to nmax (1024)
// with a prime factor above 11, which the LDS kernels would run as
// direct-sum stages (primes up to 256) or as their own Bluestein convolution
// (larger primes); measured faster than both on every length tried.  Returns the
// convolution length (a power of two >= 2n - 1), or 0 for the other paths.
// IBP_REG_BLUESTEIN=0 turns it off (comparison runs).
int reg_bluestein_length(const FftPlan& fp, int n, int nmax) {
  if (!(fp.blu || fp.any) || n > nmax || n < 2) return 0;
  if (const char* e = getenv("IBP_REG_BLUESTEIN"))
    if (atoi(e) == 0) return 0;
  int m = 32;
  while (m < 2 * n - 1) m *= 2;
  return m;
}

// The second FP32 half spectrum, row-sum array and partial region of the
// workspace (the mixed form's direct first correction keeps the right-hand
// side's while it builds the residual's).
Cx<float>* spec32_second(const ibp_plan_s* p) {
  return p->spec32 + (size_t)p->ny * spec_plane_stride<float>(p->hp, p->nz);
}
double* rowsum_second(const ibp_plan_s* p) { return p->rowsum + (size_t)p->ny * p->nz; }
double* part_second(const ibp_plan_s* p) { return p->part + max_parts(p) * kPartStride; }

ibp_status_t check_dims(int nx, int ny, int nz, FftPlan* fpx, FftPlan* fpz) {
  switch (dims_status(nx, ny, nz, fpx, fpz)) {
    case kDimsOk: return IBP_SUCCESS;
    case kDimsInvalid: return IBP_ERROR_INVALID_VALUE;
    default: return IBP_ERROR_UNSUPPORTED_SIZE;
  }
}

// XCD map of a device: the hardware XCC ids that blocks of a wide launch
// report, numbered densely in increasing order.  Probed once per device.
struct XccMap {
  bool probed = false;
  int nq = 0;
  signed char queue[kMaxXcc];
};

hipError_t xcc_map(int device, XccMap* out) {
  static std::mutex mu;
  static std::vector<XccMap> cache;
  std::lock_guard<std::mutex> lock(mu);
  if ((int)cache.size() <= device) cache.resize(device + 1);
  XccMap& m = cache[device];
  if (!m.probed) {
    constexpr int kProbeBlocks = 4096;
    int* d = nullptr;
    std::vector<int> ids(kProbeBlocks, -1);
    hipError_t e = hipMalloc(&d, kProbeBlocks * sizeof(int));
    if (e == hipSuccess) e = launch_xcc_probe(d, kProbeBlocks, nullptr);
    if (e == hipSuccess) e = hipMemcpy(ids.data(), d, kProbeBlocks * sizeof(int), hipMemcpyDeviceToHost);
    if (d) hipFree(d);
    if (e != hipSuccess) return e;
    bool seen[kMaxXcc] = {false};
    for (int v : ids)
      if (v >= 0 && v < kMaxXcc) seen[v] = true;
    m.nq = 0;
    for (int i = 0; i < kMaxXcc; ++i) m.queue[i] = seen[i] ? (signed char)m.nq++ : (signed char)-1;
    m.probed = true;
  }
  *out = m;
  return hipSuccess;
}

bool valid_plan(const ibp_plan_s* p) { return p != nullptr && p->tables != nullptr && p->ws != nullptr; }

// Right-hand side assembled inside the first x pass (FP64 direct solve):
// f = (D u - q) * rscale is never written to memory.
struct RhsFromVelocity {
  const double *u, *v, *w, *q;
  double rscale;
};
ibp_status_t enqueue_solve(ibp_plan_s* p, const double* rhs, double* phi, hipStream_t s,
                           const RhsFromVelocity* from_u);
void purge_batch_cache(const ibp_plan_s* p);
// Tuned configurations from the tuning cache (IBP_TUNE_CACHE), if any.
void apply_cached_plan(ibp_plan_s* p);
ibp_status_t batched_or_loop(const ibp_plan_t* plans, int count, const double* const* rhs, double* const* phi,
                             hipStream_t s);

// y planes per chunk when the x/z passes run chunk by chunk on two streams
// (IBP_CHUNK planes, rounded up to whole x-pass blocks; off by default and
// for grids of fewer than three chunks).  Measured on MI355X at 512x384x512
// the chunked form is slower at every chunk size (launch granularity), so it
// is an opt-in for experiments on other shapes.
int chunk_planes(const ibp_plan_s* p) {
  int S = 0;
  if (const char* e = getenv("IBP_CHUNK")) S = atoi(e);
  if (S <= 0 || p->nz == 1) return 0;
  while (((long)S * p->nz) % p->rb64 != 0 || ((long)S * p->nz) % p->rb32 != 0) ++S;
  return p->ny >= 3 * S ? S : 0;
}

hipError_t setup_chunking(ibp_plan_s* p) {
  p->chunk = chunk_planes(p);
  if (p->chunk == 0) return hipSuccess;
  const int nch = (p->ny + p->chunk - 1) / p->chunk;
  hipError_t e = hipStreamCreateWithFlags(&p->s2, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&p->ev_fork, hipEventDisableTiming);
  for (int c = 0; c < nch && e == hipSuccess; ++c) {
    hipEvent_t a = nullptr, b = nullptr;
    e = hipEventCreateWithFlags(&a, hipEventDisableTiming);
    if (e == hipSuccess) p->ev_a.push_back(a);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b, hipEventDisableTiming);
    if (e == hipSuccess) p->ev_b.push_back(b);
  }
  return e;
}

void release(ibp_plan_s* p) {
  for (hipEvent_t e : p->ev_pool) hipEventDestroy(e);
  for (hipEvent_t e : p->ev_a) hipEventDestroy(e);
  for (hipEvent_t e : p->ev_b) hipEventDestroy(e);
  if (p->ev_fork) hipEventDestroy(p->ev_fork);
  if (p->s2) hipStreamDestroy(p->s2);
  if (p->ws_owned && p->ws) hipFree(p->ws);
  if (p->tables) hipFree(p->tables);
  if (p->helm) hipFree(p->helm);
  delete p;
}

enum Pass {
  P_XR2C, P_ZFWD, P_Y, P_ZINV, P_XC2R, P_XRES, P_CHECK, P_XRESONLY, P_XC2R_ADD, P_DIV,
  P_XZF, P_ZXI, P_ZXI_ADD, P_PROJ, P_VX, P_VZ, P_VY, P_ZERO, P_ZUP, P_XRT, P_YADD, P_COUNT
};
const char* const kPassName[P_COUNT] = {"x_r2c",  "z_fwd",      "y_solve",    "z_inv",
                                        "x_c2r",  "x_resid_r2c", "check",      "x_resid_only",
                                        "x_c2r_add", "divergence", "xz_fwd",   "zx_inv",
                                        "zx_inv_add", "projection", "visc_x", "visc_z",
                                        "visc_y", "zero_mode", "z_inv_up", "x_roundtrip",
                                        "y_solve_add"};

// Algorithmic bytes of one launch of each pass (each input element read
// once, each output element written once).  N = nx ny nz cells, Nh =
// (nx/2+1) ny nz half-spectrum coefficients of `cb` bytes (IBP_MIXED_F64INV:
// the line solve reads 8-byte and writes 16-byte coefficients, the z inverse
// and the x C2R move 16-byte ones).
double pass_bytes(const ibp_plan_s* p, int pass) {
  const double N = (double)p->nx * p->ny * p->nz;
  const double Nh = (double)p->hp * p->ny * p->nz;
  const double cb = (p->prec == IBP_FP64) ? 16.0 : 8.0;
  const bool up = p->prec == IBP_MIXED_F64INV;
  switch (pass) {
    case P_XR2C: return 8.0 * N + cb * Nh;
    case P_Y: return up ? 24.0 * Nh : 2.0 * cb * Nh;
    case P_ZINV: return up ? 32.0 * Nh : 2.0 * cb * Nh;
    case P_ZFWD: return 2.0 * cb * Nh;
    case P_XC2R: return (up ? 16.0 : cb) * Nh + 8.0 * N;
    case P_XRES: return 16.0 * N + cb * Nh;        // f and phi in, spectrum out
    case P_XRESONLY: return 16.0 * N;
    case P_XC2R_ADD: return (up ? 16.0 : cb) * Nh + 16.0 * N;    // spectrum and phi in, phi out
    case P_DIV: return 32.0 * N;                   // u, v, w in, f out
    case P_XZF: return 8.0 * N + cb * Nh;          // fused: the spectrum makes one trip
    case P_ZXI: return cb * Nh + 8.0 * N;
    case P_ZXI_ADD: return cb * Nh + 16.0 * N;
    case P_PROJ: return 72.0 * N;                  // phi, u, v, w, p in; u, v, w, p out
    case P_VX:
    case P_VZ:
    case P_VY: return 16.0 * N;                    // the field in and out
    case P_ZUP: return 24.0 * Nh;                  // FP32 spectrum in, FP64 out
    case P_XRT: return 24.0 * Nh + 8.0 * N;        // FP64 spectrum and f in, FP32 spectrum out
    case P_YADD: return 40.0 * Nh;                 // FP32 in, FP64 read and written
    default: return 0.0;
  }
}

hipError_t prof_mark(ibp_plan_s* p, int pass, hipStream_t s, bool begin) {
  if (!p->profiling) return hipSuccess;
  if (begin) {
    const size_t need = 2 * (p->ev_used + 1);
    while (p->ev_pool.size() < need) {
      hipEvent_t e;
      hipError_t err = hipEventCreate(&e);
      if (err != hipSuccess) return err;
      p->ev_pool.push_back(e);
    }
    if (p->ev_pass.size() < p->ev_used + 1) p->ev_pass.resize(p->ev_used + 1);
    p->ev_pass[p->ev_used] = pass;
    return hipEventRecord(p->ev_pool[2 * p->ev_used], s);
  }
  hipError_t err = hipEventRecord(p->ev_pool[2 * p->ev_used + 1], s);
  p->ev_used++;
  return err;
}

}  // namespace

namespace {

// LU of one direction's line operator, shared by every line of that
// direction.  Rows (lo_i, di_i, up_i): lo_i multiplies x_{i-1} and up_i
// x_{i+1}; in a cyclic matrix lo_0 multiplies x_{n-1} and up_{n-1} x_0.
// A cyclic matrix is split as B + u v^T (Sherman-Morrison) with gamma =
// -di_0, u = (gamma, 0.., up_{n-1}), v = (1, 0.., lo_0 / gamma); B is
// factored by Thomas and B^-1 u folds into w = B^-1 u / (1 + v.B^-1 u), so
// that x = y - w (y_0 + g y_{n-1}) with y = B^-1 d and g = lo_0 / gamma.
// Appends the four padded tables of `L` to `buf` and fills `d`.
void pack_line(ibp_plan_s::LineDir& d, const LineLu& L, int P, int K, std::vector<double>& buf) {
  d.P = P;
  d.K = K;
  d.n = (int)L.m.size();
  d.cyclic = L.cyclic;
  d.g = L.g;
  d.npad = (long)P * K;
  d.off = (long)buf.size();
  // zero-padded to P K rows, chunk-row major: entry i P + p is row p K + i
  std::vector<std::vector<double>> padded;
  for (const std::vector<double>* v : {&L.m, &L.s, &L.t, &L.w}) {
    std::vector<double> pad(d.npad, 0.0);
    for (int r = 0; r < d.n; ++r) pad[(long)(r % K) * P + r / K] = (*v)[r];
    buf.insert(buf.end(), pad.begin(), pad.end());
    padded.push_back(pad);
  }
  // Multipliers of the lane scans, step by step: the product of m (forward)
  // or t (backward) over the rows that lane p's running composite covers
  // before each step, composed in the kernels' order.
  const int S = P == 64 ? 6 : 5;
  std::vector<double> mu(P, 1.0), T(P, 1.0), mf((size_t)S * P), mb((size_t)S * P);
  for (int p = 0; p < P; ++p) {
    for (int i = 0; i < K; ++i) mu[p] = padded[0][(size_t)i * P + p] * mu[p];
    for (int i = K - 1; i >= 0; --i) T[p] = padded[2][(size_t)i * P + p] * T[p];
  }
  for (int st = 0, off = 1; off < P; ++st, off <<= 1) {
    std::vector<double> mu2 = mu, T2 = T;
    for (int p = 0; p < P; ++p) {
      mf[(size_t)st * P + p] = mu[p];
      mb[(size_t)st * P + p] = T[p];
      if (p >= off) mu2[p] = mu[p] * mu[p - off];
      if (p + off < P) T2[p] = T[p] * T[p + off];
    }
    mu = mu2;
    T = T2;
  }
  buf.insert(buf.end(), mf.begin(), mf.end());
  buf.insert(buf.end(), mb.begin(), mb.end());
}

}  // namespace

extern "C" {

ibp_status_t ibp_check_dims(int nx, int ny, int nz) {
  try {
    return check_dims(nx, ny, nz, nullptr, nullptr);
  } catch (...) {
    return IBP_ERROR_INTERNAL;
  }
}

const char* ibp_status_string(ibp_status_t s) {
  switch (s) {
    case IBP_SUCCESS: return "IBP_SUCCESS";
    case IBP_ERROR_INVALID_VALUE: return "IBP_ERROR_INVALID_VALUE";
    case IBP_ERROR_UNSUPPORTED_SIZE: return "IBP_ERROR_UNSUPPORTED_SIZE";
    case IBP_ERROR_OUT_OF_MEMORY: return "IBP_ERROR_OUT_OF_MEMORY";
    case IBP_ERROR_HIP: return "IBP_ERROR_HIP";
    case IBP_ERROR_INTERNAL: return "IBP_ERROR_INTERNAL";
  }
  return "IBP_UNKNOWN_STATUS";
}

int ibp_version(void) { return kVersion; }

ibp_status_t ibp_plan_create(ibp_plan_t* out, int nx, int ny, int nz, double Lx, double Lz,
                             const double* y) {
  if (out == nullptr) return IBP_ERROR_INVALID_VALUE;
  *out = nullptr;
  try {
    FftPlan fpx{}, fpz{};
    ibp_status_t st = check_dims(nx, ny, nz, &fpx, &fpz);
    if (st != IBP_SUCCESS) return st;
    if (!(std::isfinite(Lx) && Lx > 0.0 && std::isfinite(Lz) && Lz > 0.0)) return IBP_ERROR_INVALID_VALUE;
    if (y == nullptr) return IBP_ERROR_INVALID_VALUE;
    for (int j = 0; j <= ny; ++j)
      if (!std::isfinite(y[j])) return IBP_ERROR_INVALID_VALUE;
    for (int j = 0; j < ny; ++j)
      if (!(y[j + 1] > y[j])) return IBP_ERROR_INVALID_VALUE;

    ibp_plan_s* p = new (std::nothrow) ibp_plan_s;
    if (!p) return IBP_ERROR_OUT_OF_MEMORY;
    p->nx = nx;
    p->ny = ny;
    p->nz = nz;
    p->h = nx % 2 ? nx : nx / 2;   // x transform length (odd nx: the whole row, no split)
    p->hp = nx / 2 + 1;
    p->Lx = Lx;
    p->Lz = Lz;
    p->dx = Lx / nx;
    p->dz = Lz / nz;
    p->fpx = fpx;
    p->fpz = fpz;
    // x: the whole row of nx points (two rows per line); fpx is the plan of
    // the general kernels' transform length (nx/2 pairs, or nx when odd)
    p->xbm = reg_bluestein_length(fpx, nx, 1024);
    p->zbm = nz > 1 ? reg_bluestein_length(fpz, nz, 1024) : 0;
    ytri_shape(ny, &p->yP, &p->yK);
    p->xfast = rfft::supported(p->h);
    p->zfast = rfft::supported(nz);
    const long nrows = (long)ny * nz;
    p->xsmall = x_small(p->fpx, p->h);
    p->xwide = fft_wide(p->fpx);
    p->zwide = fft_wide(p->fpz);
    set_x_split(p);
    // Fused persistent x/z passes: opt-in (IBP_FUSED=1).  Measured on MI355X
    // at 512x384x512 they move the same HBM bytes as the separate passes
    // (a plane's intermediate does not stay in its XCD's L2) and run slower.
    p->fused = false;
    if (const char* e = getenv("IBP_FUSED")) p->fused = atoi(e) != 0 && p->xfast && p->zfast && fused_supported(p->h, nz);
    if (p->fused) p->nbf = nrows / fused_x_rows(p->h);
    p->zsmall = z_small(p->fpz, nz);
    set_z_split(p, 1);

    // ---- FP64 geometry of the y operator (staggered, Neumann walls)
    // face coefficients a_j, c_j; the diagonal -(a_j + c_j) is never formed:
    // the kernels use the flux-difference form of the operator.
    std::vector<double> dyf(ny), yc(ny), dyc(ny + 1, 0.0), a(ny, 0.0), c(ny, 0.0);
    for (int j = 0; j < ny; ++j) {
      dyf[j] = y[j + 1] - y[j];
      yc[j] = 0.5 * (y[j] + y[j + 1]);
    }
    for (int j = 1; j < ny; ++j) dyc[j] = yc[j] - yc[j - 1];
    for (int j = 0; j < ny; ++j) p->dyf_sum += dyf[j];
    for (int j = 0; j < ny; ++j) {
      if (j > 0) a[j] = 1.0 / (dyf[j] * dyc[j]);
      if (j < ny - 1) c[j] = 1.0 / (dyf[j] * dyc[j + 1]);
    }
    p->ya_host = a;
    p->yc_host = c;
    p->dyf_host = dyf;
    p->dyc_host = dyc;
    p->lnorm = operator_inf_norm(p, a, c);
    // ---- closed-form eigenvalues of the periodic second differences
    const long double pi = 3.141592653589793238462643383279502884L;
    std::vector<double> lx(p->hp), lz(nz);
    for (int k = 0; k < p->hp; ++k) {
      const long double sn = sinl(pi * k / nx);
      lx[k] = (double)(-4.0L * sn * sn / ((long double)p->dx * p->dx));
    }
    for (int k = 0; k < nz; ++k) {
      const long double sn = sinl(pi * k / nz);
      lz[k] = (double)(-4.0L * sn * sn / ((long double)p->dz * p->dz));
    }
    std::vector<double> twxr, twxi, twzr, twzi;
    twiddles(nx, twxr, twxi);
    twiddles(nz, twzr, twzi);

    // ---- one device allocation for all tables
    std::vector<char> host;
    auto put = [&](const void* src, size_t bytes) {
      const size_t off = host.size();
      host.resize(off + align256(bytes), 0);
      std::memcpy(host.data() + off, src, bytes);
      return off;
    };
    std::vector<float> f32;
    auto tof = [&](const std::vector<double>& v) {
      f32.assign(v.begin(), v.end());
      return put(f32.data(), f32.size() * sizeof(float));
    };
    std::vector<double> cx64(2 * (size_t)nx), cz64(2 * (size_t)nz);
    std::vector<float> cx32(2 * (size_t)nx), cz32(2 * (size_t)nz);
    for (int e = 0; e < nx; ++e) {
      cx64[2 * e] = twxr[e];
      cx64[2 * e + 1] = twxi[e];
      cx32[2 * e] = (float)twxr[e];
      cx32[2 * e + 1] = (float)twxi[e];
    }
    for (int e = 0; e < nz; ++e) {
      cz64[2 * e] = twzr[e];
      cz64[2 * e + 1] = twzi[e];
      cz32[2 * e] = (float)twzr[e];
      cz32[2 * e + 1] = (float)twzi[e];
    }
    // face coefficients zero-padded to the line solve's P*K rows
    const int ypad = p->yP * p->yK > ny ? p->yP * p->yK : ny;
    a.resize(ypad, 0.0);
    c.resize(ypad, 0.0);
    const size_t o_ya = put(a.data(), ypad * sizeof(double));
    const size_t o_yc = put(c.data(), ypad * sizeof(double));
    const size_t o_dyf = put(dyf.data(), ny * sizeof(double));
    const size_t o_dyc = put(dyc.data(), (ny + 1) * sizeof(double));
    const size_t o_lx = put(lx.data(), lx.size() * sizeof(double));
    const size_t o_lz = put(lz.data(), lz.size() * sizeof(double));
    const size_t o_twx = put(cx64.data(), cx64.size() * sizeof(double));
    const size_t o_twz = put(cz64.data(), cz64.size() * sizeof(double));
    const size_t o_ya32 = tof(a);
    const size_t o_yc32 = tof(c);
    const size_t o_lx32 = tof(lx);
    const size_t o_lz32 = tof(lz);
    const size_t o_twx32 = put(cx32.data(), cx32.size() * sizeof(float));
    const size_t o_twz32 = put(cz32.data(), cz32.size() * sizeof(float));
    // Bluestein tables: chirp, filter transform, length-m twiddles; FP64 and FP32
    size_t o_bx[6] = {0, 0, 0, 0, 0, 0}, o_bz[6] = {0, 0, 0, 0, 0, 0}, o_bxr[6] = {0, 0, 0, 0, 0, 0};
    auto put_blu = [&](const FftPlan& fp, size_t* o) {
      std::vector<double> ch, bh, twr, twi;
      bluestein_tables(fp.n, fp.m, ch, bh);
      twiddles(fp.m, twr, twi);
      std::vector<double> tw(2 * (size_t)fp.m);
      for (int e = 0; e < fp.m; ++e) {
        tw[2 * e] = twr[e];
        tw[2 * e + 1] = twi[e];
      }
      o[0] = put(ch.data(), ch.size() * sizeof(double));
      o[1] = put(bh.data(), bh.size() * sizeof(double));
      o[2] = put(tw.data(), tw.size() * sizeof(double));
      o[3] = tof(ch);
      o[4] = tof(bh);
      o[5] = tof(tw);
    };
    if (p->fpx.blu) put_blu(p->fpx, o_bx);
    if (p->fpz.blu) put_blu(p->fpz, o_bz);
    if (p->xbm) {   // the register Bluestein x tables, beside the general kernels'
      FftPlan b{};
      b.n = nx;
      b.m = p->xbm;
      put_blu(b, o_bxr);
    }
    if (p->zbm) {   // every z transform of such a plan takes the register path: same slots
      FftPlan b{};
      b.n = nz;
      b.m = p->zbm;
      put_blu(b, o_bz);
    }

    hipError_t e = hipGetDevice(&p->device);
    if (e == hipSuccess && p->fused) {
      int cus = 0, b64 = 0, b32 = 0;
      e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, p->device);
      if (e == hipSuccess) e = fused_blocks_per_cu<double>(p->h, &b64);
      if (e == hipSuccess) e = fused_blocks_per_cu<float>(p->h, &b32);
      if (const char* v = getenv("IBP_FUSED_BPCU")) {   // tuning override
        const int o = atoi(v);
        if (o > 0) {
          b64 = o < b64 ? o : b64;
          b32 = o < b32 ? o : b32;
        }
      }
      p->fblocks64 = cus * b64;
      p->fblocks32 = cus * b32;
      XccMap xm;
      if (e == hipSuccess) e = xcc_map(p->device, &xm);
      if (e == hipSuccess) {
        p->nq = xm.nq;
        for (int i = 0; i < kMaxXcc; ++i) p->xcc_queue[i] = xm.queue[i];
        if (p->nq < 1 || p->fblocks64 < p->nq || p->fblocks32 < p->nq) p->fused = false;
      }
    }
    if (e == hipSuccess) e = hipMalloc(&p->tables, host.size());
    if (e == hipSuccess) e = hipMemcpy(p->tables, host.data(), host.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      if (p->tables) hipFree(p->tables);
      delete p;
      return from_hip(e);
    }
    char* d = static_cast<char*>(p->tables);
    p->ya = reinterpret_cast<const double*>(d + o_ya);
    p->yc = reinterpret_cast<const double*>(d + o_yc);
    p->dyf = reinterpret_cast<const double*>(d + o_dyf);
    p->dyc = reinterpret_cast<const double*>(d + o_dyc);
    p->lamx = reinterpret_cast<const double*>(d + o_lx);
    p->lamz = reinterpret_cast<const double*>(d + o_lz);
    p->twx = reinterpret_cast<const Cx<double>*>(d + o_twx);
    p->twz = reinterpret_cast<const Cx<double>*>(d + o_twz);
    p->ya32 = reinterpret_cast<const float*>(d + o_ya32);
    p->yc32 = reinterpret_cast<const float*>(d + o_yc32);
    p->lamx32 = reinterpret_cast<const float*>(d + o_lx32);
    p->lamz32 = reinterpret_cast<const float*>(d + o_lz32);
    p->twx32 = reinterpret_cast<const Cx<float>*>(d + o_twx32);
    for (int t = 0; t < 3; ++t) {
      if (p->fpx.blu) {
        p->bx64[t] = reinterpret_cast<const Cx<double>*>(d + o_bx[t]);
        p->bx32[t] = reinterpret_cast<const Cx<float>*>(d + o_bx[3 + t]);
      }
      if (p->xbm) {
        p->bxr64[t] = reinterpret_cast<const Cx<double>*>(d + o_bxr[t]);
        p->bxr32[t] = reinterpret_cast<const Cx<float>*>(d + o_bxr[3 + t]);
      }
      if (p->fpz.blu || p->zbm) {
        p->bz64[t] = reinterpret_cast<const Cx<double>*>(d + o_bz[t]);
        p->bz32[t] = reinterpret_cast<const Cx<float>*>(d + o_bz[3 + t]);
      }
    }
    p->twz32 = reinterpret_cast<const Cx<float>*>(d + o_twz32);

    p->ws_bytes = workspace_bytes(p);
    e = hipMalloc(&p->ws, p->ws_bytes);
    if (e != hipSuccess) {
      hipFree(p->tables);
      delete p;
      return from_hip(e);
    }
    p->ws_owned = true;
    carve_workspace(p);
    e = setup_chunking(p);
    if (e == hipSuccess) e = reset_counters(p);
    if (e != hipSuccess) {
      release(p);
      return from_hip(e);
    }
    apply_cached_plan(p);
    *out = p;
    return IBP_SUCCESS;
  } catch (...) {
    return IBP_ERROR_INTERNAL;
  }
}

ibp_status_t ibp_plan_destroy(ibp_plan_t p) {
  if (p == nullptr) return IBP_SUCCESS;
  try {
    purge_batch_cache(p);
    release(p);
    return IBP_SUCCESS;
  } catch (...) {
    return IBP_ERROR_INTERNAL;
  }
}

ibp_status_t ibp_plan_set_precision(ibp_plan_t p, ibp_precision_t prec, double rtol, int max_iters) {
  if (!valid_plan(p)) return IBP_ERROR_INVALID_VALUE;
  if (prec != IBP_FP64 && prec != IBP_MIXED && prec != IBP_MIXED_F64SWEEP && prec != IBP_MIXED_F64INV)
    return IBP_ERROR_INVALID_VALUE;
  if (prec != IBP_FP64) {
    if (!(rtol > 0.0) || !std::isfinite(rtol)) return IBP_ERROR_INVALID_VALUE;
    if (max_iters < 0 || max_iters > 64) return IBP_ERROR_INVALID_VALUE;
    p->rtol = rtol;
    p->max_iters = max_iters;
  }
  p->prec = prec;
  ++p->gen;
  try {
    apply_cached_plan(p);
  } catch (...) {
    return IBP_ERROR_INTERNAL;
  }
  return IBP_SUCCESS;
}

ibp_status_t ibp_plan_set_bc(ibp_plan_t p, ibp_bc_t lower, ibp_bc_t upper) {
  if (!valid_plan(p)) return IBP_ERROR_INVALID_VALUE;
  if ((lower != IBP_BC_NEUMANN && lower != IBP_BC_DIRICHLET) || (upper != IBP_BC_NEUMANN && upper != IBP_BC_DIRICHLET))
    return IBP_ERROR_INVALID_VALUE;
  try {
    const int ny = p->ny;
    std::vector<double> a = p->ya_host, c = p->yc_host;
    // a Dirichlet wall: phi = 0 on the wall face, half a cell from the centre
    if (lower == IBP_BC_DIRICHLET) a[0] = 1.0 / (p->dyf_host[0] * (0.5 * p->dyf_host[0]));
    if (upper == IBP_BC_DIRICHLET) c[ny - 1] = 1.0 / (p->dyf_host[ny - 1] * (0.5 * p->dyf_host[ny - 1]));
    const float a32[2] = {(float)a[0], (float)a[ny - 1]};
    const float c32[2] = {(float)c[0], (float)c[ny - 1]};
    // only the two wall rows of each table change
    hipError_t e = hipMemcpy((void*)p->ya, a.data(), sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy((void*)(p->yc + ny - 1), &c[ny - 1], sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy((void*)p->ya32, &a32[0], sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy((void*)(p->yc32 + ny - 1), &c32[1], sizeof(float), hipMemcpyHostToDevice);
    if (e != hipSuccess) return from_hip(e);
    p->bc_lo = lower;
    p->bc_hi = upper;
    p->lnorm = operator_inf_norm(p, a, c);
    ++p->gen;
    return IBP_SUCCESS;
  } catch (...) {
    return IBP_ERROR_INTERNAL;
  }
}

ibp_status_t ibp_plan_workspace_size(ibp_plan_t p, size_t* bytes) {
  if (!valid_plan(p) || bytes == nullptr) return IBP_ERROR_INVALID_VALUE;
  *bytes = workspace_bytes(p);
  return IBP_SUCCESS;
}

ibp_status_t ibp_plan_set_workspace(ibp_plan_t p, void* ptr, size_t bytes) {
  if (!valid_plan(p)) return IBP_ERROR_INVALID_VALUE;
  try {
    const size_t need = workspace_bytes(p);
    if (ptr != nullptr) {
      if ((reinterpret_cast<uintptr_t>(ptr) & 255) != 0) return IBP_ERROR_INVALID_VALUE;
      if (bytes < need) return IBP_ERROR_OUT_OF_MEMORY;
      if (p->ws_owned) hipFree(p->ws);
      p->ws = ptr;
      p->ws_bytes = bytes;
      p->ws_owned = false;
    } else {
      void* w = nullptr;
      hipError_t e = hipMalloc(&w, need);
      if (e != hipSuccess) return from_hip(e);
      if (p->ws_owned) hipFree(p->ws);
      p->ws = w;
      p->ws_bytes = need;
      p->ws_owned = true;
    }
    carve_workspace(p);
    ++p->gen;
    return from_hip(reset_counters(p));
  } catch (...) {
    return IBP_ERROR_INTERNAL;
  }
}

ibp_status_t ibp_solve(ibp_plan_t p, const double* rhs, double* phi, hipStream_t stream) {
  if (!valid_plan(p) || rhs == nullptr || phi == nullptr) return IBP_ERROR_INVALID_VALUE;
  if ((reinterpret_cast<uintptr_t>(rhs) & 15) != 0 || (reinterpret_cast<uintptr_t>(phi) & 15) != 0)
    return IBP_ERROR_INVALID_VALUE;
  const size_t n = (size_t)p->nx * p->ny * p->nz;
  if (p->prec != IBP_FP64) {
    const uintptr_t r0 = reinterpret_cast<uintptr_t>(rhs), r1 = r0 + n * sizeof(double);
    const uintptr_t q0 = reinterpret_cast<uintptr_t>(phi), q1 = q0 + n * sizeof(double);
    if (r0 < q1 && q0 < r1) return IBP_ERROR_INVALID_VALUE;
  }
  try {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return from_hip(e);
    if (dev != p->device) return IBP_ERROR_INVALID_VALUE;
    roctxRangePushA("ibp_solve");
    const ibp_status_t st = enqueue_solve(p, rhs, phi, static_cast<hipStream_t>(stream), nullptr);
    roctxRangePop();
    return st;
  } catch (...) {
    return IBP_ERROR_INTERNAL;
  }
}

ibp_status_t ibp_solve_batched(const ibp_plan_t* plans, int count, const double* const* rhs,
                               double* const* phi, hipStream_t stream) {
  if (count < 0) return IBP_ERROR_INVALID_VALUE;
  if (count == 0) return IBP_SUCCESS;
  if (plans == nullptr || rhs == nullptr || phi == nullptr) return IBP_ERROR_INVALID_VALUE;
  for (int i = 0; i < count; ++i) {
    if (!valid_plan(plans[i]) || rhs[i] == nullptr || phi[i] == nullptr) return IBP_ERROR_INVALID_VALUE;
    for (int k = 0; k < i; ++k)
      if (plans[k] == plans[i]) return IBP_ERROR_INVALID_VALUE;
  }
  try {
    return batched_or_loop(plans, count, rhs, phi, static_cast<hipStream_t>(stream));
  } catch (...) {
    return IBP_ERROR_INTERNAL;
  }
}

ibp_status_t ibp_get_info(ibp_plan_t p, ibp_info_t* out) {
  if (!valid_plan(p) || out == nullptr) return IBP_ERROR_INVALID_VALUE;
  try {
    std::memset(out, 0, sizeof(*out));
    if (!p->solved) {
      out->rel_residual = NAN;
      out->rel_residual_vw = NAN;
      out->backward_error = NAN;
      return IBP_SUCCESS;
    }
    hipError_t e = hipStreamSynchronize(p->last_stream);
    Ctl c{};
    const Ctl* src = p->info_ctl ? p->info_ctl : p->ctl;
    if (e == hipSuccess) e = hipMemcpy(&c, src, sizeof(Ctl), hipMemcpyDeviceToHost);
    int dep_error = 0;
    if (e == hipSuccess) e = hipMemcpy(&dep_error, p->fctl + kFctlError, sizeof(int), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return from_hip(e);
    if (dep_error) {   // a fused pass gave up waiting on a dependency: results invalid
      hipMemset(p->fctl + kFctlError, 0, sizeof(int));
      return IBP_ERROR_INTERNAL;
    }
    out->iterations = c.iters;
    out->converged = c.converged;
    out->nonfinite_input = c.nonfinite;
    out->rel_residual = c.rel_residual;
    out->removed_mean = c.removed_mean;
    out->rhs_norm = std::sqrt(c.fnorm2);
    out->residual_norm = std::sqrt(c.rnorm2);
    out->rel_residual_vw = c.rel_residual_vw;
    out->backward_error = c.backward_error;
    out->history_len = std::min(std::max(c.nhist, 0), std::min(kHistMax, IBP_HISTORY_MAX));
    for (int k = 0; k < out->history_len; ++k) out->residual_history[k] = c.hist[k];
    return IBP_SUCCESS;
  } catch (...) {
    return IBP_ERROR_INTERNAL;
  }
}

ibp_status_t ibp_plan_set_profiling(ibp_plan_t p, int enable) {
  if (!valid_plan(p)) return IBP_ERROR_INVALID_VALUE;
  p->profiling = enable != 0;
  p->ev_used = 0;
  return IBP_SUCCESS;
}

ibp_status_t ibp_plan_get_profile(ibp_plan_t p, int max, int* count, ibp_pass_stat_t* stats) {
  if (!valid_plan(p) || count == nullptr || (max > 0 && stats == nullptr) || max < 0) return IBP_ERROR_INVALID_VALUE;
  try {
    double ms[P_COUNT] = {0};
    int n[P_COUNT] = {0};
    for (size_t i = 0; i < p->ev_used; ++i) {
      hipError_t e = hipEventSynchronize(p->ev_pool[2 * i + 1]);
      float t = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&t, p->ev_pool[2 * i], p->ev_pool[2 * i + 1]);
      if (e != hipSuccess) return from_hip(e);
      ms[p->ev_pass[i]] += t;
      n[p->ev_pass[i]] += 1;
    }
    p->ev_used = 0;
    int c = 0;
    for (int k = 0; k < P_COUNT; ++k) {
      if (n[k] == 0) continue;
      if (c < max) {
        std::memset(&stats[c], 0, sizeof(ibp_pass_stat_t));
        std::strncpy(stats[c].name, kPassName[k], sizeof(stats[c].name) - 1);
        stats[c].launches = n[k];
        stats[c].total_ms = ms[k];
        stats[c].bytes_per_launch = pass_bytes(p, k);
      }
      ++c;
    }
    *count = c < max ? c : max;
    return IBP_SUCCESS;
  } catch (...) {
    return IBP_ERROR_INTERNAL;
  }
}

ibp_status_t ibp_divergence(ibp_plan_t p, const double* u, const double* v, const double* w, double* f,
                            hipStream_t stream) {
  if (!valid_plan(p) || !u || !v || !w || !f) return IBP_ERROR_INVALID_VALUE;
  try {
    DivArgs a{u, v, w, nullptr, f, p->dyf, p->nx, p->ny, p->nz, 1.0 / p->dx, 1.0 / p->dz, 1.0};
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = prof_mark(p, P_DIV, s, true);
    if (e == hipSuccess) e = launch_divergence(a, s);
    if (e == hipSuccess) e = prof_mark(p, P_DIV, s, false);
    return from_hip(e);
  } catch (...) {
    return IBP_ERROR_INTERNAL;
  }
}

namespace {
bool aligned16(const void* ptr) { return (reinterpret_cast<uintptr_t>(ptr) & 15) == 0; }
}  // namespace

ibp_status_t ibp_solve_divergence(ibp_plan_t p, const double* u, const double* v, const double* w, const double* q,
                                  double alpha_dt, double* rhs_out, double* phi, hipStream_t stream) {
  if (!valid_plan(p) || !u || !v || !w || !phi) return IBP_ERROR_INVALID_VALUE;
  if (!(alpha_dt > 0.0) || !std::isfinite(alpha_dt)) return IBP_ERROR_INVALID_VALUE;
  if (!aligned16(u) || !aligned16(v) || !aligned16(w) || !aligned16(phi) || (q && !aligned16(q)) ||
      (rhs_out && !aligned16(rhs_out)))
    return IBP_ERROR_INVALID_VALUE;
  if (p->prec != IBP_FP64 && rhs_out == nullptr) return IBP_ERROR_INVALID_VALUE;   // refinement re-reads f
  try {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return from_hip(e);
    if (dev != p->device) return IBP_ERROR_INVALID_VALUE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (rhs_out == nullptr) {   // FP64: assembled inside the first x pass
      RhsFromVelocity r{u, v, w, q, 1.0 / alpha_dt};
      return enqueue_solve(p, nullptr, phi, s, &r);
    }
    DivArgs a{u, v, w, q, rhs_out, p->dyf, p->nx, p->ny, p->nz, 1.0 / p->dx, 1.0 / p->dz, 1.0 / alpha_dt};
    e = prof_mark(p, P_DIV, s, true);
    if (e == hipSuccess) e = launch_divergence(a, s);
    if (e == hipSuccess) e = prof_mark(p, P_DIV, s, false);
    if (e != hipSuccess) return from_hip(e);
    return ibp_solve(p, rhs_out, phi, stream);
  } catch (...) {
    return IBP_ERROR_INTERNAL;
  }
}

ibp_status_t ibp_project(ibp_plan_t p, const double* phi, double alpha_dt, double visc, double* u, double* v,
                         double* w, double* pr, hipStream_t stream) {
  if (!valid_plan(p) || !phi || !u || !v || !w) return IBP_ERROR_INVALID_VALUE;
  if (!std::isfinite(alpha_dt) || !std::isfinite(visc)) return IBP_ERROR_INVALID_VALUE;
  try {
    ProjArgs a{phi, u, v, w, pr, p->dyf, p->dyc, p->ya, p->yc, p->nx, p->ny, p->nz,
               p->bc_lo == IBP_BC_DIRICHLET ? 1 : 0, p->bc_hi == IBP_BC_DIRICHLET ? 1 : 0,
               1.0 / p->dx, 1.0 / p->dz, alpha_dt, visc};
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = prof_mark(p, P_PROJ, s, true);
    if (e == hipSuccess) e = launch_project(a, s);
    if (e == hipSuccess) e = prof_mark(p, P_PROJ, s, false);
    return from_hip(e);
  } catch (...) {
    return IBP_ERROR_INTERNAL;
  }
}

ibp_status_t ibp_helmholtz_set(ibp_plan_t p, double beta) {
  if (!valid_plan(p)) return IBP_ERROR_INVALID_VALUE;
  if (!(beta >= 0.0) || !std::isfinite(beta)) return IBP_ERROR_INVALID_VALUE;
  try {
    const int nx = p->nx, ny = p->ny, nz = p->nz;
    int Px, Kx, Pz, Kz, Pc, Kc, Pf = 32, Kf = 2;
    if (!line_shape(nx, &Px, &Kx) || !line_shape(nz, &Pz, &Kz) || !line_shape(ny, &Pc, &Kc))
      return IBP_ERROR_UNSUPPORTED_SIZE;
    const bool faces = p->bc_lo == IBP_BC_NEUMANN && p->bc_hi == IBP_BC_NEUMANN && ny >= 2;
    if (faces && !line_shape(ny - 1, &Pf, &Kf)) return IBP_ERROR_UNSUPPORTED_SIZE;
    std::vector<double> buf;
    ibp_plan_s::LineDir hx, hz, hyc, hyf;
    {   // periodic second differences along x and z
      const double rx = beta / (p->dx * p->dx), rz = beta / (p->dz * p->dz);
      pack_line(hx, line_lu(std::vector<double>(nx, -rx), std::vector<double>(nx, 1.0 + 2.0 * rx),
                            std::vector<double>(nx, -rx), true), Px, Kx, buf);
      pack_line(hz, line_lu(std::vector<double>(nz, -rz), std::vector<double>(nz, 1.0 + 2.0 * rz),
                            std::vector<double>(nz, -rz), true), Pz, Kz, buf);
    }
    {   // cell centres: velocity prescribed where the plan's wall is Neumann
      std::vector<double> a = p->ya_host, c = p->yc_host, lo(ny), di(ny), up(ny);
      const std::vector<double>& dyf = p->dyf_host;
      a[0] = p->bc_lo == IBP_BC_NEUMANN ? 1.0 / (dyf[0] * (0.5 * dyf[0])) : 0.0;
      c[ny - 1] = p->bc_hi == IBP_BC_NEUMANN ? 1.0 / (dyf[ny - 1] * (0.5 * dyf[ny - 1])) : 0.0;
      for (int j = 0; j < ny; ++j) {
        lo[j] = -beta * a[j];
        up[j] = -beta * c[j];
        di[j] = 1.0 + beta * (a[j] + c[j]);
      }
      pack_line(hyc, line_lu(lo, di, up, false), Pc, Kc, buf);
    }
    if (faces) {   // interior y faces 1..ny-1, wall faces held at zero
      const int n = ny - 1;
      std::vector<double> lo(n), di(n), up(n);
      for (int r = 0; r < n; ++r) {
        const int j = r + 1;
        const double l = 1.0 / (p->dyc_host[j] * p->dyf_host[j - 1]);
        const double u = 1.0 / (p->dyc_host[j] * p->dyf_host[j]);
        lo[r] = -beta * l;
        up[r] = -beta * u;
        di[r] = 1.0 + beta * (l + u);
      }
      pack_line(hyf, line_lu(lo, di, up, false), Pf, Kf, buf);
    }
    if (buf.size() > p->helm_doubles) {
      if (p->helm) hipFree(p->helm);
      p->helm = nullptr;
      p->helm_doubles = 0;
      p->helm_ready = false;
      hipError_t e = hipMalloc((void**)&p->helm, buf.size() * sizeof(double));
      if (e != hipSuccess) return from_hip(e);
      p->helm_doubles = buf.size();
    }
    hipError_t e = hipMemcpy(p->helm, buf.data(), buf.size() * sizeof(double), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      p->helm_ready = false;
      return from_hip(e);
    }
    p->hx = hx;
    p->hz = hz;
    p->hyc = hyc;
    p->hyf = hyf;
    p->helm_faces = faces;
    p->helm_lo = p->bc_lo;
    p->helm_hi = p->bc_hi;
    p->helm_ready = true;
    return IBP_SUCCESS;
  } catch (...) {
    return IBP_ERROR_INTERNAL;
  }
}

ibp_status_t ibp_helmholtz(ibp_plan_t p, double* field, ibp_location_t where, hipStream_t stream) {
  if (!valid_plan(p) || field == nullptr || !aligned16(field)) return IBP_ERROR_INVALID_VALUE;
  if (where != IBP_AT_CELLS && where != IBP_AT_YFACES) return IBP_ERROR_INVALID_VALUE;
  if (!p->helm_ready || p->helm_lo != p->bc_lo || p->helm_hi != p->bc_hi) return IBP_ERROR_INVALID_VALUE;
  if (where == IBP_AT_YFACES && !p->helm_faces) return IBP_ERROR_INVALID_VALUE;
  try {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return from_hip(e);
    if (dev != p->device) return IBP_ERROR_INVALID_VALUE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const long plane = (long)p->nx * p->nz;
    const bool cells = where == IBP_AT_CELLS;
    const int planes = cells ? p->ny : p->ny - 1;
    double* base = cells ? field : field + plane;
    const ibp_plan_s::LineDir& hy = cells ? p->hyc : p->hyf;
    LineArgs ax{base, p->helm + p->hx.off, p->hx.npad, p->nx, p->hx.cyclic, p->hx.g, 0, 0, (long)planes * p->nz, 0};
    // the z lines run in descending block order: the x pass wrote the last
    // planes last, and they are still in the Infinity Cache
    LineArgs az{base, p->helm + p->hz.off, p->hz.npad, p->nz, p->hz.cyclic, p->hz.g, planes, plane, p->nx, p->nx, 1};
    LineArgs ay{base, p->helm + hy.off, hy.npad, planes, 0, 0.0, 1, 0, plane, plane};
    if (!cells) {   // the increment vanishes on the wall faces
      e = launch_fill_zero(field, plane, s);
      if (e == hipSuccess) e = launch_fill_zero(field + (long)p->ny * plane, plane, s);
      if (e != hipSuccess) return from_hip(e);
    }
    e = prof_mark(p, P_VX, s, true);
    if (e == hipSuccess) e = launch_lines_contig(p->hx.P, p->hx.K, ax, s);
    if (e == hipSuccess) e = prof_mark(p, P_VX, s, false);
    if (e == hipSuccess) e = prof_mark(p, P_VZ, s, true);
    if (e == hipSuccess) e = launch_lines_strided(p->hz.P, p->hz.K, az, s);
    if (e == hipSuccess) e = prof_mark(p, P_VZ, s, false);
    if (e == hipSuccess) e = prof_mark(p, P_VY, s, true);
    if (e == hipSuccess) e = launch_lines_strided(hy.P, hy.K, ay, s);
    if (e == hipSuccess) e = prof_mark(p, P_VY, s, false);
    return from_hip(e);
  } catch (...) {
    return IBP_ERROR_INTERNAL;
  }
}

}  // extern "C"

namespace {

// LDS Bluestein z transforms (lines the register path does not take):
// column stride m + 1 and the tables.
template <typename T>
void zf_bluestein(const ibp_plan_s* p, ZfArgs<T>& z) {
  if (!p->fpz.blu || p->zbm) return;
  z.zss = p->fpz.m + 1;
  if constexpr (sizeof(T) == 8) {
    z.bc = p->bz64[0]; z.bb = p->bz64[1]; z.bt = p->bz64[2];
  } else {
    z.bc = p->bz32[0]; z.bb = p->bz32[1]; z.bt = p->bz32[2];
  }
}

template <typename T>
XArgs<T> xargs(ibp_plan_s* p, const double* rhs, const double* phi_in, double* phi_out, Cx<T>* spec,
               const Cx<T>* twx, int rb, int iter) {
  XArgs<T> a{};
  a.f = rhs;
  a.phi = phi_in;
  a.out = phi_out;
  a.spec = spec;
  a.rowsum = p->rowsum;
  a.part = p->part;
  a.phi00 = p->phi00;
  a.ctl = p->ctl;
  a.twx = twx;
  a.ya = p->ya;
  a.yc = p->yc;
  a.dyf = p->dyf;
  a.fp = p->fpx;
  a.nx = p->nx;
  a.ny = p->ny;
  a.nz = p->nz;
  a.h = p->h;
  a.hp = p->hp;
  a.rs = spec_row_stride<T>(p->hp);
  a.ps = spec_plane_stride<T>(p->hp, p->nz);
  a.rows_per_block = rb;
  a.row_begin = 0;
  a.nrows = (long)p->ny * p->nz;
  a.parts = 1;
  a.idx2 = 1.0 / (p->dx * p->dx);
  a.idz2 = 1.0 / (p->dz * p->dz);
  a.out_scale = 1.0 / ((double)p->h * (double)p->nz);
  a.inv_nxnz = 1.0 / ((double)p->nx * (double)p->nz);
  a.iter = iter;
  if (p->fpx.blu) {
    a.hs = p->fpx.m;
    if constexpr (sizeof(T) == 8) {
      a.bc = p->bx64[0]; a.bb = p->bx64[1]; a.bt = p->bx64[2];
    } else {
      a.bc = p->bx32[0]; a.bb = p->bx32[1]; a.bt = p->bx32[2];
    }
  }
  return a;
}

ZeroArgs zargs(ibp_plan_s* p, long nparts, int init, int mixed, int iter, int final_pass) {
  ZeroArgs z{};
  z.rowsum = p->rowsum;
  z.ghat = p->ghat;
  z.ticket = p->ticket;
  z.phi00 = p->phi00;
  z.dyf = p->dyf;
  z.dyc = p->dyc;
  z.part = p->part;
  z.part2 = p->part + 2 * max_parts(p) * kPartStride;
  z.nparts = nparts;
  z.ctl = p->ctl;
  z.nx = p->nx;
  z.ny = p->ny;
  z.nz = p->nz;
  z.init = init;
  z.mixed = mixed;
  z.iter = iter;
  z.final_pass = final_pass;
  z.rtol = p->rtol;
  z.dyf_sum = p->dyf_sum;
  z.singular = p->singular();
  z.lnorm = p->lnorm;
  return z;
}

// Launch `call` on `strm` with optional profiling events around it.
// Each launch is also a roctx range named after its pass (visible to
// rocprofv3 --marker-trace; a no-op without a profiler).
#define IBP_LAUNCH_ON(pass, strm, ...)                         \
  do {                                                         \
    roctxRangePushA(kPassName[(pass)]);                        \
    hipError_t e_ = prof_mark(p, (pass), (strm), true);        \
    if (e_ == hipSuccess) e_ = (__VA_ARGS__);                  \
    if (e_ == hipSuccess) e_ = prof_mark(p, (pass), (strm), false); \
    roctxRangePop();                                           \
    if (e_ != hipSuccess) return from_hip(e_);                 \
  } while (0)
#define IBP_LAUNCH(pass, ...) IBP_LAUNCH_ON(pass, s, __VA_ARGS__)
#define IBP_HIP(...)                                  \
  do {                                                \
    hipError_t e_ = (__VA_ARGS__);                    \
    if (e_ != hipSuccess) return from_hip(e_);        \
  } while (0)

// The register Bluestein x path's arguments: its own tables (whole rows of
// nx points), kept apart from the LDS kernels' Bluestein tables.
template <typename T>
XArgs<T> with_xblu(const ibp_plan_s* p, const XArgs<T>& a) {
  XArgs<T> b = a;
  if constexpr (sizeof(T) == 8) {
    b.bc = p->bxr64[0]; b.bb = p->bxr64[1]; b.bt = p->bxr64[2];
  } else {
    b.bc = p->bxr32[0]; b.bb = p->bxr32[1]; b.bt = p->bxr32[2];
  }
  return b;
}

template <typename T>
hipError_t run_xr2c(const ibp_plan_s* p, int mode, const XArgs<T>& a, hipStream_t s) {
  if (p->xfast && mode != XM_RESID_ONLY) return launch_xr2c_fast<T>(mode, a, s);
  // register Bluestein: the FP64 right-hand side pass (the others keep the
  // LDS kernels, whose norm partials and residual modes it does not carry)
  if constexpr (sizeof(T) == 8)
    if (p->xbm && mode == XM_PLAIN && p->chunk <= 0) return launch_xblu_r2c<T>(with_xblu(p, a), p->xbm, s);
  if (mode == XM_RESID_ONLY) {
    XArgs<T> b = a;
    b.row_begin = 0;
    b.nrows = (long)p->ny * p->nz;
    if constexpr (sizeof(T) == 4)
      if (resid_march_blocks(p->nx, p->ny, p->nz) > 0) return launch_resid_march(b, s);
    b.rows_per_block = x_tile_rows(p, x_tile32(p));
    b.parts = 1;
    return launch_xr2c<T>(mode, p->xsmall, p->xwide, b, s);
  }
  return launch_xr2c<T>(mode, p->xsmall, p->xwide, a, s);
}

template <typename T>
hipError_t run_xc2r(const ibp_plan_s* p, int mode, const XArgs<T>& a, hipStream_t s) {
  if (p->xfast) return launch_xc2r_fast<T>(mode, a, s);
  if (p->xbm && p->chunk <= 0) return launch_xblu_c2r<T>(mode, with_xblu(p, a), p->xbm, s);
  return launch_xc2r<T>(mode, p->xsmall, p->xwide, a, s);
}

template <typename T>
hipError_t run_zfft(const ibp_plan_s* p, bool inverse, const ZfArgs<T>& a, int nplanes, hipStream_t s) {
  if (p->zfast) return launch_zfft_fast<T>(inverse, a, nplanes, s);
  if (p->zbm) {
    ZfArgs<T> b = a;
    if constexpr (sizeof(T) == 8) {
      b.bc = p->bz64[0]; b.bb = p->bz64[1]; b.bt = p->bz64[2];
    } else {
      b.bc = p->bz32[0]; b.bb = p->bz32[1]; b.bt = p->bz32[2];
    }
    return launch_zblu_reg<T>(inverse, b, p->zbm, nplanes, s);
  }
  return launch_zfft<T>(inverse, p->zsmall, p->zwide, a, nplanes, s);
}

// Forward transforms of the whole grid: x R2C then z FFT.  With chunking,
// the two passes run plane chunk by plane chunk, the z pass of chunk c on
// the plan's second stream right after the x pass of chunk c, so a chunk's
// half spectrum is still resident in the Infinity Cache when the z pass
// reads it; at most two chunks are in flight.
template <typename T>
FusedArgs<T> fused_args(const ibp_plan_s* p, const XArgs<T>& xa, const ZfArgs<T>& za, bool fwd) {
  FusedArgs<T> F{};
  F.x = xa;
  F.x.row_begin = 0;
  F.x.nrows = (long)p->ny * p->nz;
  F.z = za;
  F.z.plane0 = 0;
  F.queue = p->fctl + kFctlQueue;
  F.exit_count = p->fctl + kFctlExit;
  F.error = p->fctl + kFctlError;
  F.done = p->fctl + kFctlHead;
  F.nq = p->nq;
  for (int i = 0; i < kMaxXcc; ++i) F.xcc_queue[i] = p->xcc_queue[i];
  const int nx_items = p->nz / fused_x_rows(p->h);
  const int nz_items = (p->hp + fused_z_cols(p->nz) - 1) / fused_z_cols(p->nz);
  F.nfirst = fwd ? nx_items : nz_items;
  F.nsecond = fwd ? nz_items : nx_items;
  F.ny = p->ny;
  const int G = (sizeof(T) == 8 ? p->fblocks64 : p->fblocks32) / p->nq;   // blocks per XCD
  // lag: rounds between a plane's first-stage and second-stage items, so
  // that the blocks in flight on one XCD rarely wait on a dependency
  int lag = (G + F.nfirst + F.nsecond - 1) / (F.nfirst + F.nsecond) + 1;
  if (const char* e = getenv("IBP_FUSED_LAG")) lag = atoi(e) > 0 ? atoi(e) : lag;
  F.lag = lag < 1 ? 1 : lag;
  return F;
}

template <typename T>
ibp_status_t forward_xz(ibp_plan_s* p, XArgs<T> xa, int xmode, int xpass, ZfArgs<T> za, hipStream_t s) {
  const int ny = p->ny, nz = p->nz, S = p->chunk;
  if (p->fused && xmode == XM_PLAIN && S <= 0) {
    const int G = sizeof(T) == 8 ? p->fblocks64 : p->fblocks32;
    IBP_LAUNCH(P_XZF, launch_fused_fwd<T>(fused_args<T>(p, xa, za, true), G, s));
    return IBP_SUCCESS;
  }
  if (S <= 0 || nz == 1) {
    xa.row_begin = 0;
    xa.nrows = (long)ny * nz;
    IBP_LAUNCH(xpass, run_xr2c<T>(p, xmode, xa, s));
    za.plane0 = 0;
    if (nz > 1) IBP_LAUNCH(P_ZFWD, run_zfft<T>(p, false, za, ny, s));
    return IBP_SUCCESS;
  }
  hipStream_t s2 = p->s2;
  const int nch = (ny + S - 1) / S;
  IBP_HIP(hipEventRecord(p->ev_fork, s));
  IBP_HIP(hipStreamWaitEvent(s2, p->ev_fork, 0));
  for (int c = 0; c < nch; ++c) {
    const int j0 = c * S, j1 = j0 + S < ny ? j0 + S : ny;
    if (c >= 2) IBP_HIP(hipStreamWaitEvent(s, p->ev_b[c - 2], 0));
    xa.row_begin = (long)j0 * nz;
    xa.nrows = (long)j1 * nz;
    IBP_LAUNCH_ON(xpass, s, run_xr2c<T>(p, xmode, xa, s));
    IBP_HIP(hipEventRecord(p->ev_a[c], s));
    IBP_HIP(hipStreamWaitEvent(s2, p->ev_a[c], 0));
    za.plane0 = j0;
    IBP_LAUNCH_ON(P_ZFWD, s2, run_zfft<T>(p, false, za, j1 - j0, s2));
    IBP_HIP(hipEventRecord(p->ev_b[c], s2));
  }
  IBP_HIP(hipStreamWaitEvent(s, p->ev_b[nch - 1], 0));
  return IBP_SUCCESS;
}

// Inverse transforms: z inverse FFT then x C2R, chunked the same way (z on
// the second stream, x on the caller's stream).
template <typename T>
ibp_status_t inverse_zx(ibp_plan_s* p, XArgs<T> xa, int cmode, int xpass, ZfArgs<T> za, hipStream_t s) {
  const int ny = p->ny, nz = p->nz, S = p->chunk;
  if (p->fused && S <= 0 && (cmode == CM_SET || sizeof(T) == 4)) {
    const int G = sizeof(T) == 8 ? p->fblocks64 : p->fblocks32;
    IBP_LAUNCH(cmode == CM_SET ? P_ZXI : P_ZXI_ADD, launch_fused_inv<T>(cmode, fused_args<T>(p, xa, za, false), G, s));
    return IBP_SUCCESS;
  }
  if (S <= 0 || nz == 1) {
    za.plane0 = 0;
    if (nz > 1) IBP_LAUNCH(P_ZINV, run_zfft<T>(p, true, za, ny, s));
    xa.row_begin = 0;
    xa.nrows = (long)ny * nz;
    IBP_LAUNCH(xpass, run_xc2r<T>(p, cmode, xa, s));
    return IBP_SUCCESS;
  }
  hipStream_t s2 = p->s2;
  const int nch = (ny + S - 1) / S;
  IBP_HIP(hipEventRecord(p->ev_fork, s));
  IBP_HIP(hipStreamWaitEvent(s2, p->ev_fork, 0));
  for (int c = 0; c < nch; ++c) {
    const int j0 = c * S, j1 = j0 + S < ny ? j0 + S : ny;
    if (c >= 2) IBP_HIP(hipStreamWaitEvent(s2, p->ev_a[c - 2], 0));
    za.plane0 = j0;
    IBP_LAUNCH_ON(P_ZINV, s2, run_zfft<T>(p, true, za, j1 - j0, s2));
    IBP_HIP(hipEventRecord(p->ev_b[c], s2));
    IBP_HIP(hipStreamWaitEvent(s, p->ev_b[c], 0));
    xa.row_begin = (long)j0 * nz;
    xa.nrows = (long)j1 * nz;
    IBP_LAUNCH_ON(xpass, s, run_xc2r<T>(p, cmode, xa, s));
    IBP_HIP(hipEventRecord(p->ev_a[c], s));
  }
  return IBP_SUCCESS;
}

template <typename U>
ibp_status_t enqueue_mixed(ibp_plan_s* p, const double* rhs, double* phi, hipStream_t s, bool f64inv);

ibp_status_t enqueue_solve(ibp_plan_s* p, const double* rhs, double* phi, hipStream_t s,
                           const RhsFromVelocity* from_u) {
  p->last_stream = s;
  p->solved = true;
  p->info_ctl = p->ctl;
  if (p->prec == IBP_MIXED) return enqueue_mixed<float>(p, rhs, phi, s, false);
  if (p->prec == IBP_MIXED_F64SWEEP) return enqueue_mixed<double>(p, rhs, phi, s, false);
  if (p->prec == IBP_MIXED_F64INV) return enqueue_mixed<double>(p, rhs, phi, s, true);
  // FP64 direct solve: x R2C, z FFT, y line solves + FP64 (0,0), z inverse, x C2R
  XArgs<double> xa = xargs<double>(p, rhs, nullptr, phi, p->spec64, p->twx, p->rb64, 0);
  xa.parts = 0;   // no norms needed: non-finite input shows up in the FP64 plane sums
  int xmode = XM_PLAIN;
  if (from_u) {
    xmode = XM_DIV;
    xa.u = from_u->u;
    xa.v = from_u->v;
    xa.w = from_u->w;
    xa.q = from_u->q;
    xa.idx = 1.0 / p->dx;
    xa.idz = 1.0 / p->dz;
    xa.rscale = from_u->rscale;
  }
  ZfArgs<double> za{p->spec64, p->twz, p->ctl, p->fpz, p->nz, p->hp, p->zc64,
                    spec_row_stride<double>(p->hp), spec_plane_stride<double>(p->hp, p->nz), 0, 0};
  zf_bluestein(p, za);
  ibp_status_t st = forward_xz<double>(p, xa, xmode, P_XR2C, za, s);
  if (st != IBP_SUCCESS) return st;
  YArgs<double, double> ya{p->spec64, p->lamx, p->lamz, p->ya, p->yc, p->ctl,
                           (long)p->nz * spec_row_stride<double>(p->hp), spec_row_stride<double>(p->hp),
                           spec_plane_stride<double>(p->hp, p->nz), p->ny, p->hp, 0, p->singular()};
  IBP_LAUNCH(P_Y, launch_ytri<double, double>(p->yP, p->yK, p->ycols, ya, zargs(p, 0, 1, 0, 0, 0), s));
  return inverse_zx<double>(p, xa, CM_SET, P_XC2R, za, s);
}

// FP64 inverse passes of IBP_MIXED_F64INV: the FP64 z inverse and x C2R (set
// or add into phi) on the FP64 half spectrum the line solve wrote.
ibp_status_t inverse_f64(ibp_plan_s* p, const double* rhs, double* phi, int cmode, int iter, int check_done,
                         hipStream_t s) {
  ZfArgs<double> za{p->spec64, p->twz, p->ctl, p->fpz, p->nz, p->hp, p->zc64,
                    spec_row_stride<double>(p->hp), spec_plane_stride<double>(p->hp, p->nz), check_done, 0};
  zf_bluestein(p, za);
  if (p->nz > 1) IBP_LAUNCH(P_ZINV, run_zfft<double>(p, true, za, p->ny, s));
  XArgs<double> xd = xargs<double>(p, rhs, phi, phi, p->spec64, p->twx, p->rb64, iter);
  xd.parts = 0;
  IBP_LAUNCH(cmode == CM_SET ? P_XC2R : P_XC2R_ADD, run_xc2r<double>(p, cmode, xd, s));
  return IBP_SUCCESS;
}

// IBP_MIXED_F64INV on the register kernels (power-of-two x and z lengths
// in their fused range), unchunked, with at least one correction allowed:
// the first correction is computed without forming the initial iterate.
bool direct_first_correction(const ibp_plan_s* p) {
  const bool hx = p->h >= 32 && p->h <= 512 && p->nx == 2 * p->h;
  const bool hz = p->nz >= 32 && p->nz <= 1024;
  return p->xfast && p->zfast && hx && hz && !p->fused && p->chunk <= 0 && p->max_iters >= 1;
}

// Mixed forms: FP32 spectral passes wrapped in FP64 iterative refinement.
//   pass 0: phi = solve32(f)                      (rows summed in FP64 for (0,0))
//   pass k: r = f - m - L_h phi (FP64), stop if ||r|| <= rtol ||f - m||,
//           else phi += solve32(r * s_k) / s_k   (s_k a power of two)
//   final : residual of the last iterate.
// Every pass is enqueued; once the control block marks the solve done the
// remaining kernels return immediately.  f64inv (U = double): the line
// solve of every solve32 writes its FP64 solution to the FP64 half spectrum
// and the inverse z and x passes run in FP64 (inverse_f64).
template <typename U>
ibp_status_t enqueue_mixed(ibp_plan_s* p, const double* rhs, double* phi, hipStream_t s, bool f64inv) {
  const U* lx = nullptr;
  const U* lz = nullptr;
  const U *ca = nullptr, *cc = nullptr;
  if constexpr (sizeof(U) == 8) {
    lx = p->lamx; lz = p->lamz; ca = p->ya; cc = p->yc;
  } else {
    lx = p->lamx32; lz = p->lamz32; ca = p->ya32; cc = p->yc32;
  }
  const long rs = spec_row_stride<float>(p->hp), ps = spec_plane_stride<float>(p->hp, p->nz);
  const long Q = (long)p->nz * rs;
  ZfArgs<float> za{p->spec32, p->twz32, p->ctl, p->fpz, p->nz, p->hp, p->zc32, rs, ps, 0, 0};
  zf_bluestein(p, za);
  YArgs<float, U> ya{p->spec32, lx, lz, ca, cc, p->ctl, Q, rs, ps, p->ny, p->hp, 0, p->singular()};

  XArgs<float> xa = xargs<float>(p, rhs, phi, phi, p->spec32, p->twx32, p->rb32, 0);
  ibp_status_t st = forward_xz<float>(p, xa, XM_PLAIN, P_XR2C, za, s);
  if (st != IBP_SUCCESS) return st;
  // partials of the initial pass: one per x-row block of whichever x kernel ran
  const long np0 = (p->fused && p->chunk <= 0) ? p->nbf : p->nb32;
  if constexpr (sizeof(U) == 8) {
    ya.out64 = p->spec64;
    ya.out_rs = spec_row_stride<double>(p->hp);
    ya.out_ps = spec_plane_stride<double>(p->hp, p->nz);
  }
  auto ysolve = [&](const ZeroArgs& z) {
    if constexpr (sizeof(U) == 8) {
      if (f64inv) return launch_ytri_out64(p->yP, p->yK, ya, z, s);
    }
    return launch_ytri<float, U>(p->yP, p->yK, p->ycols, ya, z, s);
  };
  int k0 = 1;   // first refinement pass of the loop below
  if (f64inv && direct_first_correction(p)) {
    // The initial iterate phi_0 = IFFT64(solve(F32)) is never formed: its
    // residual is f - IFFT64(F32) (the rounding of the FP32 forward
    // transform; the line solve and the FP64 inverse add only FP64
    // rounding), so the first correction is solved from that and the two
    // solutions are added in the spectrum, inverted once.  (0,0) mode of a
    // singular problem: taken from the FP64 row sums as in every pass, so
    // r0 drops the FP32 spectrum's (0,0) coefficient and subtracts the exact
    // plane means instead.
    ZeroArgs z0 = zargs(p, np0, 1, 1, 0, 0);
    IBP_LAUNCH(P_ZERO, launch_zero_mode(z0, s));   // solve control, mean, (0,0) mode of f
    const long rs64 = spec_row_stride<double>(p->hp), ps64 = spec_plane_stride<double>(p->hp, p->nz);
    ZupArgs zu{p->spec32, rs, ps, p->spec64, rs64, ps64, p->twz, p->nz, p->hp, p->ny, p->singular() ? 1 : 0};
    IBP_LAUNCH(P_ZUP, launch_zinv_up(zu, s));
    RtArgs rt{};
    rt.x = xargs<float>(p, rhs, phi, phi, spec32_second(p), p->twx32, p->rb32, 1);
    rt.x.row_begin = 0;
    rt.x.nrows = (long)p->ny * p->nz;
    rt.x.rowsum = rowsum_second(p);
    rt.x.part = part_second(p);
    rt.t64 = p->spec64;
    rt.trs = rs64;
    rt.tps = ps64;
    rt.twx64 = p->twx;
    rt.ghat = p->ghat;
    rt.sub_mean = p->singular() ? 1 : 0;
    IBP_LAUNCH(P_XRT, launch_x_roundtrip(rt, s));
    // the right-hand side's line solve (its (0,0) mode was solved above)
    IBP_LAUNCH(P_Y, ysolve(zargs(p, np0, 0, 1, 0, 0)));
    // record the residual of phi_0 and prepare the correction (never stops:
    // the solution is not formed yet)
    ZeroArgs zc = zargs(p, p->nb32, 0, 1, 1, 0);
    zc.part = part_second(p);
    zc.nostop = 1;
    IBP_LAUNCH(P_CHECK, launch_check(zc, s));
    // the correction, added to the FP64 spectrum and to the (0,0) mode
    ZfArgs<float> zr = za;
    zr.spec = spec32_second(p);
    zr.plane0 = 0;
    IBP_LAUNCH(P_ZFWD, run_zfft<float>(p, false, zr, p->ny, s));
    YArgs<float, U> yr = ya;
    yr.spec = spec32_second(p);
    yr.add_iter = 1;
    ZeroArgs zy = zargs(p, p->nb32, 0, 1, 1, 0);
    zy.rowsum = rowsum_second(p);
    zy.phi00_add = 1;
    if constexpr (sizeof(U) == 8) IBP_LAUNCH(P_YADD, launch_ytri_out64(p->yP, p->yK, yr, zy, s));
    st = inverse_f64(p, rhs, phi, CM_SET, 1, 0, s);
    if (st != IBP_SUCCESS) return st;
    k0 = 2;
  } else {
    IBP_LAUNCH(P_Y, ysolve(zargs(p, np0, 1, 1, 0, 0)));
    st = f64inv ? inverse_f64(p, rhs, phi, CM_SET, 0, 0, s) : inverse_zx<float>(p, xa, CM_SET, P_XC2R, za, s);
    if (st != IBP_SUCCESS) return st;
  }

  za.check_done = 1;
  ya.check_done = 1;
  for (int k = k0; k <= p->max_iters; ++k) {
    xa.iter = k;
    // the residual pass is not chunked: the convergence test needs all of it
    xa.row_begin = 0;
    xa.nrows = (long)p->ny * p->nz;
    if (k >= 2) {   // residual-only probe of the corrected iterate (runs when predicted to converge)
      XArgs<float> xp = xa;
      xp.probe = 1;
      IBP_LAUNCH(P_XRESONLY, run_xr2c<float>(p, XM_RESID_ONLY, xp, s));
      ZeroArgs zp = zargs(p, p->nbro, 0, 1, k, 0);
      zp.probe = 1;
      IBP_LAUNCH(P_CHECK, launch_check(zp, s));
    }
    IBP_LAUNCH(P_XRES, run_xr2c<float>(p, XM_RESID, xa, s));
    IBP_LAUNCH(P_CHECK, launch_check(zargs(p, p->nb32, 0, 1, k, 0), s));
    ZfArgs<float> zf = za;
    zf.plane0 = 0;
    if (p->nz > 1) IBP_LAUNCH(P_ZFWD, run_zfft<float>(p, false, zf, p->ny, s));
    IBP_LAUNCH(P_Y, ysolve(zargs(p, p->nb32, 0, 1, k, 0)));
    st = f64inv ? inverse_f64(p, rhs, phi, CM_ADD, k, 1, s) : inverse_zx<float>(p, xa, CM_ADD, P_XC2R_ADD, za, s);
    if (st != IBP_SUCCESS) return st;
  }
  xa.iter = p->max_iters + 1;
  IBP_LAUNCH(P_XRESONLY, run_xr2c<float>(p, XM_RESID_ONLY, xa, s));
  IBP_LAUNCH(P_CHECK, launch_check(zargs(p, p->nbro, 0, 1, p->max_iters + 1, 1), s));
  return IBP_SUCCESS;
}

}  // namespace

// ======================================================================
// Batches: many uneven grids solved together, one launch per stage that
// covers every grid.  Per-grid arguments sit in a device table built once;
// the line-solve coefficient tables are re-padded to the batch's common
// lanes x rows shape (the largest ny decides it).
struct ibp_batch_s {
  int device = 0;
  int count = 0;
  ibp_precision_t prec = IBP_FP64;
  int max_iters = 0;
  std::vector<ibp_plan_t> plans;
  std::vector<unsigned> gens;
  void* dmem = nullptr;
  void* desc = nullptr;      // BatchGrid<T>[count]
  long* start = nullptr;     // [7][count + 1]: prefix offsets of the stage launches (nblk order)
  // blocks of the x (narrow, wide family), z (narrow, wide) and y (rows per
  // lane K, K/2, K/4) stage launches: each stage runs as several launches
  // over the grids of one kind (a grid has no blocks in the others)
  long nblk[7] = {0, 0, 0, 0, 0, 0, 0};
  int yKc[3] = {0, 0, 0}, yMc[3] = {0, 0, 0};   // rows per lane and columns per block of the y launches
  int yP = 32, yK = 2, yM = 8;
  int xdiv = 1, zdiv = 1;    // x rows and z columns per block: the largest tile's, divided by these
  bool zsmall = false;       // every grid's z lines fit the small tile
  bool xsmall = false;       // every grid's x rows fit the small tile
  std::vector<long> hstart;
  std::vector<int> rbmax, zcmax;   // per grid: rows per block and z columns of the largest tile
  std::vector<BatchGrid<double>> h64;
  std::vector<BatchGrid<float>> h32;
  // persistent schedule: the whole solve in one launch (ibp_persist.hip)
  bool persist_ok = false;   // small tiles and a line-solve shape the persistent kernel is built for
  bool persist = false;      // solve with it
  bool wide = false;         // some grid needs the wide transform family
  int persist_blocks = 0;    // blocks of the persistent launch
  int lag = 1;               // diagonal interleave of the grids' stages in a queue
  int smax = 0;              // stages per grid (counters per grid)
  void* pmem = nullptr;      // segments | queue offsets | items per queue | claim heads | counters | exit count
  PersistArgs pargs{};
};

namespace {

constexpr int kBatchDivMax = 4;   // finest x split the partial buffers are sized for

// Apply the batch's work split (x rows per block, z columns per block, line-
// solve columns per block) to the per-grid arguments and prefix offsets and
// upload them (synchronous).  The split changes which block does what, not
// the arithmetic: results are bitwise the same for every split.
template <typename T>
hipError_t persist_schedule(ibp_batch_s* b, const std::vector<BatchGrid<T>>& hd);

template <typename T>
hipError_t batch_apply(ibp_batch_s* b, std::vector<BatchGrid<T>>& hd) {
  const int n = b->count;
  b->hstart.assign(7 * (n + 1), 0);
  long* h[7];
  for (int i = 0; i < 7; ++i) h[i] = b->hstart.data() + i * (n + 1);
  // y launches: the base shape's K, K/2, K/4 rows per lane, with columns per
  // block raised in proportion (same LDS tile, same bytes per block)
  for (int c = 0; c < 3; ++c) {
    const bool ok = b->yK % (1 << c) == 0;
    b->yKc[c] = ok ? b->yK >> c : 0;
    const int want = b->yM << c < 16 ? b->yM << c : 16;
    b->yMc[c] = ok ? batch_ytri_cols<T>(b->yP, b->yKc[c], want) : 0;
  }
  for (int g = 0; g < n; ++g) {
    BatchGrid<T>& d = hd[g];
    const int rb = b->rbmax[g] / b->xdiv > 0 ? b->rbmax[g] / b->xdiv : 1;
    const int zc = b->zcmax[g] / b->zdiv > 0 ? b->zcmax[g] / b->zdiv : 1;
    const long nxb = (d.x.nrows + rb - 1) / rb;
    d.x.rows_per_block = rb;
    if (d.x.parts) d.zero.nparts = nxb;
    d.z.cols = zc;
    d.zcolblocks = (d.z.hp + zc - 1) / zc;
    const long nzb = d.z.nz > 1 ? (long)d.zcolblocks * d.y.ny : 0;
    const bool xw = b->plans[g]->xwide, zw = b->plans[g]->zwide;
    h[0][g + 1] = h[0][g] + (xw ? 0 : nxb);
    h[1][g + 1] = h[1][g] + (xw ? nxb : 0);
    h[2][g + 1] = h[2][g] + (zw ? 0 : nzb);
    h[3][g + 1] = h[3][g] + (zw ? nzb : 0);
    for (int c = 0; c < 3; ++c) {
      const int M = b->yMc[c];
      h[4 + c][g + 1] = h[4 + c][g] + (d.yk == b->yKc[c] ? (d.y.Q + M - 1) / M + zero_blocks(d.y.ny) : 0);
    }
  }
  for (int i = 0; i < 7; ++i) b->nblk[i] = h[i][n];
  hipError_t e = hipMemcpy(b->desc, hd.data(), n * sizeof(BatchGrid<T>), hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(b->start, b->hstart.data(), b->hstart.size() * sizeof(long), hipMemcpyHostToDevice);
  if (e == hipSuccess && b->persist_ok) e = persist_schedule<T>(b, hd);
  return e;
}

// The per-XCD work queues of the persistent schedule for the current work
// split.  Stages of one grid run in order, each waiting for the previous
// one to complete; a grid's stages all go to one queue (grids dealt to the
// queues by decreasing size, each to the least loaded).  In a queue the
// segments follow diagonals: stage s of the i-th grid has key s + lag i.
template <typename T>
hipError_t persist_schedule(ibp_batch_s* b, const std::vector<BatchGrid<T>>& hd) {
  const int n = b->count;
  const bool mixed = b->prec == IBP_MIXED;
  const int M = kThreads / b->yP;
  struct St {
    int kind, iter, flags;
    long count;
  };
  std::vector<std::vector<St>> stages(n);
  std::vector<double> work(n, 0.0);
  for (int g = 0; g < n; ++g) {
    const BatchGrid<T>& d = hd[g];
    const long nxb = (d.x.nrows + d.x.rows_per_block - 1) / d.x.rows_per_block;
    const long nzb = d.z.nz > 1 ? (long)d.zcolblocks * d.y.ny : 0;
    const long nyb = (d.y.Q + M - 1) / M + zero_blocks(d.y.ny);
    const int yk = d.yk == b->yK ? PK_Y0 : (d.yk == b->yK / 2 ? PK_Y1 : PK_Y2);
    auto& v = stages[g];
    v.push_back({PK_XR2C, 0, 0, nxb});
    v.push_back({PK_ZF, 0, 0, nzb});
    v.push_back({yk, 0, PF_INIT, nyb});
    v.push_back({PK_ZI, 0, 0, nzb});
    v.push_back({PK_XC2R, 0, 0, nxb});
    if (mixed) {
      for (int k = 1; k <= b->max_iters; ++k) {
        v.push_back({PK_XRES, k, 0, nxb});
        v.push_back({PK_CHECK, k, 0, 1});
        v.push_back({PK_ZF, k, PF_CHECK_DONE, nzb});
        v.push_back({yk, k, PF_CHECK_DONE, nyb});
        v.push_back({PK_ZI, k, PF_CHECK_DONE, nzb});
        v.push_back({PK_XC2R_ADD, k, 0, nxb});
      }
      v.push_back({PK_XRESONLY, b->max_iters + 1, 0, nxb});
      v.push_back({PK_CHECK, b->max_iters + 1, PF_FINAL, 1});
    }
    v.erase(std::remove_if(v.begin(), v.end(), [](const St& x) { return x.count == 0; }), v.end());
    work[g] = (double)b->plans[g]->nx * b->plans[g]->ny * b->plans[g]->nz;
  }
  const int nq = b->pargs.nq;
  const std::vector<std::vector<int>> qgrids = lpt_queues(work, nq);
  std::vector<PersistSeg> segs;
  std::vector<int> qseg(nq + 1, 0);
  std::vector<long> qitems(nq, 0);
  for (int q = 0; q < nq; ++q) {
    qseg[q] = (int)segs.size();
    std::vector<int> nstages;
    for (int g : qgrids[q]) nstages.push_back((int)stages[g].size());
    long first = 0;
    for (const DiagItem& k : diagonal_order(nstages, b->lag)) {
      const int g = qgrids[q][k.pos];
      const St& x = stages[g][k.stage];
      PersistSeg sg{};
      sg.first = first;
      sg.g = g;
      sg.kind = x.kind;
      sg.iter = x.iter;
      sg.flags = x.flags;
      sg.done = g * b->smax + k.stage;
      sg.dep = k.stage > 0 ? g * b->smax + k.stage - 1 : -1;
      sg.need = k.stage > 0 ? (int)stages[g][k.stage - 1].count : 0;
      segs.push_back(sg);
      first += x.count;
    }
    qitems[q] = first;
  }
  qseg[nq] = (int)segs.size();
  // device layout: segments | qseg | qitems (sized for the largest schedule at build)
  char* base = static_cast<char*>(b->pmem);
  const size_t o_qseg = align256((size_t)b->count * b->smax * sizeof(PersistSeg));
  const size_t o_qitems = o_qseg + align256((kMaxXcc + 1) * sizeof(int));
  hipError_t e = hipMemcpy(base, segs.data(), segs.size() * sizeof(PersistSeg), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(base + o_qseg, qseg.data(), qseg.size() * sizeof(int), hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(base + o_qitems, qitems.data(), qitems.size() * sizeof(long), hipMemcpyHostToDevice);
  return e;
}

hipError_t batch_reapply(ibp_batch_s* b) {
  return b->prec == IBP_FP64 ? batch_apply<double>(b, b->h64) : batch_apply<float>(b, b->h32);
}

// Persistent schedule of a batch: available when every grid fits the small
// transform tiles and the line-solve shape is one the persistent kernel is
// built for (off with IBP_PERSIST=0).  Allocates the queue tables and the
// counters (zeroed here; each launch re-arms them before it ends) and sizes
// the launch to the resident blocks of the device.
template <typename T>
hipError_t persist_setup(ibp_batch_s* b) {
  b->wide = false;
  for (ibp_plan_t p : b->plans) b->wide = b->wide || p->xwide || p->zwide;
  b->persist_ok = b->xsmall && b->zsmall && persist_shape_supported(b->yP, b->yK);
  if (const char* e = getenv("IBP_PERSIST")) b->persist_ok = b->persist_ok && atoi(e) != 0;
  b->persist = false;
  if (!b->persist_ok) return hipSuccess;
  XccMap m;
  hipError_t e = xcc_map(b->device, &m);
  if (e != hipSuccess) return e;
  if (m.nq < 1 || m.nq > kMaxXcc) {
    b->persist_ok = false;
    return hipSuccess;
  }
  int per_cu = 0, ncu = 0;
  e = persist_blocks_per_cu<T>(b->wide, b->yP, b->yK, &per_cu);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, b->device);
  if (e != hipSuccess) return e;
  if (per_cu < 1 || ncu < 1) {
    b->persist_ok = false;
    return hipSuccess;
  }
  b->persist_blocks = std::max(m.nq, (per_cu * ncu) / m.nq * m.nq);
  const bool mixed = b->prec == IBP_MIXED;
  b->smax = 5 + (mixed ? 6 * b->max_iters + 2 : 0);
  const size_t nseg = (size_t)b->count * b->smax;
  const size_t o_qseg = align256(nseg * sizeof(PersistSeg));
  const size_t o_qitems = o_qseg + align256((kMaxXcc + 1) * sizeof(int));
  const size_t o_head = o_qitems + align256(kMaxXcc * sizeof(long));
  const size_t o_cnt = o_head + align256(kMaxXcc * sizeof(int));
  const size_t o_exit = o_cnt + align256(nseg * sizeof(int));
  const size_t bytes = o_exit + align256(sizeof(int));
  e = hipMalloc(&b->pmem, bytes);
  if (e == hipSuccess) e = hipMemset(b->pmem, 0, bytes);
  if (e != hipSuccess) return e;
  char* base = static_cast<char*>(b->pmem);
  PersistArgs& a = b->pargs;
  a = PersistArgs{};
  a.grids = b->desc;
  a.seg = reinterpret_cast<const PersistSeg*>(base);
  a.qseg = reinterpret_cast<const int*>(base + o_qseg);
  a.qitems = reinterpret_cast<const long*>(base + o_qitems);
  a.head = reinterpret_cast<int*>(base + o_head);
  a.cnt = reinterpret_cast<int*>(base + o_cnt);
  a.exit_count = reinterpret_cast<int*>(base + o_exit);
  a.ncnt = (int)nseg;
  a.nq = m.nq;
  a.mixed = mixed ? 1 : 0;
  a.chunk = 8;
  for (int i = 0; i < kMaxXcc; ++i) a.xcc_queue[i] = m.queue[i];
  for (int g = 0; g < b->count; ++g) a.err[g] = b->plans[g]->fctl + kFctlError;
  // measured slower than one launch per stage on the 64-grid batch (4.6 ms
  // against 2.9 ms FP64): opt-in (ibp_batch_set_persistent) or chosen by the
  // batch autotuner when it is faster
  b->persist = false;
  return hipSuccess;
}

template <typename T>
ibp_status_t batch_build(ibp_batch_s* b) {
  constexpr bool kF64 = sizeof(T) == 8;
  b->xsmall = true;
  for (ibp_plan_t p : b->plans) b->xsmall = b->xsmall && x_small(p->fpx, p->h);
  const int TLX = b->xsmall ? (kF64 ? kTileX64s : kTileX32s) : (kF64 ? kTileX64 : kTileX32);
  b->zsmall = true;
  for (ibp_plan_t p : b->plans) b->zsmall = b->zsmall && z_small(p->fpz, p->nz);
  const int TLZ = b->zsmall ? (kF64 ? kTileZ64s : kTileZ32s) : (kF64 ? kTileZ64 : kTileZ32);
  const int n = b->count;
  int maxny = 0;
  for (ibp_plan_t p : b->plans) maxny = p->ny > maxny ? p->ny : maxny;
  if (!ytri_shape(maxny, &b->yP, &b->yK)) return IBP_ERROR_UNSUPPORTED_SIZE;
  int want = 0;
  if (const char* e = getenv("IBP_YCOLS")) want = atoi(e);
  b->yM = batch_ytri_cols<T>(b->yP, b->yK, want);
  const int PK = b->yP * b->yK;
  // device memory: descriptors | prefix offsets | padded a, c tables | partials
  std::vector<size_t> o_part(n);
  const size_t o_start = align256(n * sizeof(BatchGrid<T>));
  const size_t o_tab = o_start + align256(7 * (n + 1) * sizeof(long));
  size_t bytes = o_tab + align256((size_t)n * 2 * PK * sizeof(T));
  for (int g = 0; g < n; ++g) {
    const ibp_plan_s* p = b->plans[g];
    o_part[g] = bytes;
    if (!kF64) {   // partials of the finest x split
      const long nrows = (long)p->ny * p->nz;
      const int rbmin = TLX / p->h / kBatchDivMax > 0 ? TLX / p->h / kBatchDivMax : 1;
      bytes += align256((size_t)((nrows + rbmin - 1) / rbmin) * kPartStride * sizeof(double));
    }
  }
  hipError_t e = hipMalloc(&b->dmem, bytes);
  if (e != hipSuccess) return from_hip(e);
  char* base = static_cast<char*>(b->dmem);
  b->desc = base;
  b->start = reinterpret_cast<long*>(base + o_start);
  T* dtab = reinterpret_cast<T*>(base + o_tab);
  std::vector<T> tab((size_t)n * 2 * PK, T(0));
  std::vector<BatchGrid<T>> hd(n);
  b->rbmax.assign(n, 1);
  b->zcmax.assign(n, 1);
  for (int g = 0; g < n; ++g) {
    ibp_plan_s* p = b->plans[g];
    std::vector<double> a(p->ny), c(p->ny);
    e = hipMemcpy(a.data(), p->ya, p->ny * sizeof(double), hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(c.data(), p->yc, p->ny * sizeof(double), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return from_hip(e);
    T* ta = tab.data() + (size_t)g * 2 * PK;
    T* tc = ta + PK;
    for (int j = 0; j < p->ny; ++j) {
      ta[j] = (T)a[j];
      tc[j] = (T)c[j];
    }
    BatchGrid<T>& d = hd[g];
    Cx<T>* spec;
    const Cx<T>* twx;
    const Cx<T>* twz;
    const T *lx, *lz;
    if constexpr (kF64) {
      spec = p->spec64; twx = p->twx; twz = p->twz; lx = p->lamx; lz = p->lamz;
    } else {
      spec = p->spec32; twx = p->twx32; twz = p->twz32; lx = p->lamx32; lz = p->lamz32;
    }
    b->rbmax[g] = TLX / p->h;
    int cols = TLZ / p->nz;
    if (cols > 64) cols = 64;
    if (cols > p->hp) cols = p->hp;
    b->zcmax[g] = cols;
    double* part = kF64 ? p->part : reinterpret_cast<double*>(base + o_part[g]);
    d.x = xargs<T>(p, nullptr, nullptr, nullptr, spec, twx, b->rbmax[g], 0);
    d.x.parts = kF64 ? 0 : 1;
    d.x.part = part;
    const long rs = spec_row_stride<T>(p->hp), ps = spec_plane_stride<T>(p->hp, p->nz);
    d.z = ZfArgs<T>{spec, twz, p->ctl, p->fpz, p->nz, p->hp, cols, rs, ps, 0, 0};
    d.y = YArgs<T, T>{spec, lx, lz, dtab + (size_t)g * 2 * PK, dtab + (size_t)g * 2 * PK + PK, p->ctl,
                      (long)p->nz * rs, rs, ps, p->ny, p->hp, 0, p->singular()};
    d.zero = zargs(p, 0, 0, 0, 0, 0);
    d.zero.part = part;
    d.yk = batch_grid_rows_per_lane(p->ny, b->yP, b->yK);
  }
  e = hipMemcpy(dtab, tab.data(), tab.size() * sizeof(T), hipMemcpyHostToDevice);
  if (e != hipSuccess) return from_hip(e);
  e = persist_setup<T>(b);
  if (e == hipSuccess) e = batch_apply<T>(b, hd);
  if (e != hipSuccess) return from_hip(e);
  if constexpr (kF64) b->h64 = std::move(hd); else b->h32 = std::move(hd);
  return IBP_SUCCESS;
}

template <typename T>
ibp_status_t batch_enqueue(ibp_batch_s* b, const double* const* rhs, double* const* phi, hipStream_t s) {
  const int n = b->count;
  BatchPtrs P{};
  for (int g = 0; g < n; ++g) {
    P.f[g] = rhs[g];
    P.phi[g] = phi[g];
  }
  const BatchGrid<T>* d = static_cast<const BatchGrid<T>*>(b->desc);
  const long* st[7];
  for (int i = 0; i < 7; ++i) st[i] = b->start + i * (n + 1);
  const bool mixed = b->prec == IBP_MIXED;
  for (ibp_plan_t p : b->plans) {
    p->last_stream = s;
    p->solved = true;
    p->info_ctl = p->ctl;
  }
  if (b->persist) {   // every stage of every grid in one launch
    IBP_HIP(launch_persist<T>(b->wide, b->yP, b->yK, b->pargs, P, b->persist_blocks, s));
    return IBP_SUCCESS;
  }
  // each transform stage: the narrow-family launch, then the wide one
  auto xr2c = [&](int mode, const BatchLaunch& l) {
    hipError_t e = launch_batch_xr2c<T>(mode, b->xsmall, false, d, st[0], b->nblk[0], P, l, s);
    return e == hipSuccess ? launch_batch_xr2c<T>(mode, b->xsmall, true, d, st[1], b->nblk[1], P, l, s) : e;
  };
  auto xc2r = [&](int mode, const BatchLaunch& l) {
    hipError_t e = launch_batch_xc2r<T>(mode, b->xsmall, false, d, st[0], b->nblk[0], P, l, s);
    return e == hipSuccess ? launch_batch_xc2r<T>(mode, b->xsmall, true, d, st[1], b->nblk[1], P, l, s) : e;
  };
  auto zfft = [&](bool inverse, const BatchLaunch& l) {
    hipError_t e = launch_batch_zfft<T>(inverse, b->zsmall, false, d, st[2], b->nblk[2], l, s);
    return e == hipSuccess ? launch_batch_zfft<T>(inverse, b->zsmall, true, d, st[3], b->nblk[3], l, s) : e;
  };
  auto ytri = [&](const BatchLaunch& l) {
    hipError_t e = hipSuccess;
    for (int c = 0; c < 3 && e == hipSuccess; ++c)
      if (b->nblk[4 + c] > 0) e = launch_batch_ytri<T>(b->yP, b->yKc[c], b->yMc[c], d, st[4 + c], b->nblk[4 + c], l, s);
    return e;
  };
  BatchLaunch L{n, 0, 1, mixed ? 1 : 0, 0, 0};
  IBP_HIP(xr2c(XM_PLAIN, L));
  IBP_HIP(zfft(false, L));
  IBP_HIP(ytri(L));
  IBP_HIP(zfft(true, L));
  IBP_HIP(xc2r(CM_SET, L));
  if (!mixed) return IBP_SUCCESS;
  for (int k = 1; k <= b->max_iters; ++k) {
    L = BatchLaunch{n, k, 0, 1, 0, 1};
    IBP_HIP(xr2c(XM_RESID, L));
    IBP_HIP(launch_batch_check<T>(d, L, s));
    IBP_HIP(zfft(false, L));
    IBP_HIP(ytri(L));
    IBP_HIP(zfft(true, L));
    IBP_HIP(xc2r(CM_ADD, L));
  }
  L = BatchLaunch{n, b->max_iters + 1, 0, 1, 1, 1};
  IBP_HIP(xr2c(XM_RESID_ONLY, L));
  IBP_HIP(launch_batch_check<T>(d, L, s));
  return IBP_SUCCESS;
}

ibp_status_t apply_cached_batch(ibp_batch_s* b);

void batch_free(ibp_batch_s* b) {
  if (b == nullptr) return;
  if (b->dmem) hipFree(b->dmem);
  if (b->pmem) hipFree(b->pmem);
  delete b;
}

// Checks shared by ibp_batch_create and the cached path of ibp_solve_batched.
ibp_status_t batch_eligible(const ibp_plan_t* plans, int count, int device) {
  if (count < 1 || count > kBatchMax) return IBP_ERROR_INVALID_VALUE;
  for (int i = 0; i < count; ++i) {
    if (!valid_plan(plans[i]) || plans[i]->device != device) return IBP_ERROR_INVALID_VALUE;
    for (int k = 0; k < i; ++k)
      if (plans[k] == plans[i]) return IBP_ERROR_INVALID_VALUE;
    if (plans[i]->prec != plans[0]->prec) return IBP_ERROR_INVALID_VALUE;
    if (plans[i]->prec == IBP_MIXED && plans[i]->max_iters != plans[0]->max_iters) return IBP_ERROR_INVALID_VALUE;
    // batches size every grid's general tiles whole (no direct-sum stages)
    // and split every row into pairs (even nx)
    if (plans[i]->fpx.any || plans[i]->fpz.any || plans[i]->fpx.blu || plans[i]->fpz.blu || plans[i]->nx % 2)
      return IBP_ERROR_UNSUPPORTED_SIZE;
  }
  if (plans[0]->prec != IBP_FP64 && plans[0]->prec != IBP_MIXED) return IBP_ERROR_UNSUPPORTED_SIZE;
  return IBP_SUCCESS;
}

ibp_status_t batch_create(const ibp_plan_t* plans, int count, ibp_batch_s** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return from_hip(e);
  ibp_status_t st = batch_eligible(plans, count, dev);
  if (st != IBP_SUCCESS) return st;
  ibp_batch_s* b = new (std::nothrow) ibp_batch_s;
  if (!b) return IBP_ERROR_OUT_OF_MEMORY;
  b->device = dev;
  b->count = count;
  b->prec = plans[0]->prec;
  b->max_iters = plans[0]->max_iters;
  b->plans.assign(plans, plans + count);
  for (int i = 0; i < count; ++i) b->gens.push_back(plans[i]->gen);
  st = b->prec == IBP_FP64 ? batch_build<double>(b) : batch_build<float>(b);
  if (st == IBP_SUCCESS) st = apply_cached_batch(b);
  if (st != IBP_SUCCESS) {
    batch_free(b);
    return st;
  }
  *out = b;
  return IBP_SUCCESS;
}

bool batch_current(const ibp_batch_s* b) {
  for (int i = 0; i < b->count; ++i)
    if (b->plans[i]->gen != b->gens[i]) return false;
  return true;
}

ibp_status_t batch_solve(ibp_batch_s* b, const double* const* rhs, double* const* phi, hipStream_t s) {
  if (rhs == nullptr || phi == nullptr) return IBP_ERROR_INVALID_VALUE;
  if (!batch_current(b)) return IBP_ERROR_INVALID_VALUE;
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return from_hip(e);
  if (dev != b->device) return IBP_ERROR_INVALID_VALUE;
  for (int g = 0; g < b->count; ++g) {
    if (rhs[g] == nullptr || phi[g] == nullptr) return IBP_ERROR_INVALID_VALUE;
    if ((reinterpret_cast<uintptr_t>(rhs[g]) & 15) != 0 || (reinterpret_cast<uintptr_t>(phi[g]) & 15) != 0)
      return IBP_ERROR_INVALID_VALUE;
    if (b->prec != IBP_FP64) {
      const ibp_plan_s* p = b->plans[g];
      const size_t n = (size_t)p->nx * p->ny * p->nz * sizeof(double);
      const uintptr_t r0 = reinterpret_cast<uintptr_t>(rhs[g]), q0 = reinterpret_cast<uintptr_t>(phi[g]);
      if (r0 < q0 + n && q0 < r0 + n) return IBP_ERROR_INVALID_VALUE;
    }
  }
  roctxRangePushA(b->persist ? "ibp_batch_solve_persistent" : "ibp_batch_solve_staged");
  const ibp_status_t st =
      b->prec == IBP_FP64 ? batch_enqueue<double>(b, rhs, phi, s) : batch_enqueue<float>(b, rhs, phi, s);
  roctxRangePop();
  return st;
}

// Batches built by ibp_solve_batched, keyed by the exact plan sequence.
struct BatchCacheEntry {
  std::vector<ibp_plan_t> key;
  ibp_batch_s* batch;
};
std::mutex g_batch_mu;
std::vector<BatchCacheEntry> g_batch_cache;
constexpr size_t kBatchCacheMax = 16;

void purge_batch_cache(const ibp_plan_s* p) {
  std::lock_guard<std::mutex> lock(g_batch_mu);
  for (size_t i = 0; i < g_batch_cache.size();) {
    const auto& k = g_batch_cache[i].key;
    if (std::find(k.begin(), k.end(), p) != k.end()) {
      batch_free(g_batch_cache[i].batch);
      g_batch_cache.erase(g_batch_cache.begin() + i);
    } else {
      ++i;
    }
  }
}

ibp_status_t batched_or_loop(const ibp_plan_t* plans, int count, const double* const* rhs, double* const* phi,
                             hipStream_t s) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return from_hip(e);
  bool together = count >= 2;
  for (int c0 = 0; together && c0 < count; c0 += kBatchMax) {
    const int m = count - c0 < kBatchMax ? count - c0 : kBatchMax;
    if (m >= 2 && batch_eligible(plans + c0, m, dev) != IBP_SUCCESS) together = false;
  }
  if (!together) {
    for (int i = 0; i < count; ++i) {
      ibp_status_t st = ibp_solve(plans[i], rhs[i], phi[i], s);
      if (st != IBP_SUCCESS) return st;
    }
    return IBP_SUCCESS;
  }
  for (int c0 = 0; c0 < count; c0 += kBatchMax) {
    const int m = count - c0 < kBatchMax ? count - c0 : kBatchMax;
    if (m == 1) {
      ibp_status_t st = ibp_solve(plans[c0], rhs[c0], phi[c0], s);
      if (st != IBP_SUCCESS) return st;
      continue;
    }
    ibp_batch_s* b = nullptr;
    {
      std::lock_guard<std::mutex> lock(g_batch_mu);
      std::vector<ibp_plan_t> key(plans + c0, plans + c0 + m);
      for (size_t i = 0; i < g_batch_cache.size(); ++i) {
        if (g_batch_cache[i].key == key) {
          if (batch_current(g_batch_cache[i].batch)) {
            b = g_batch_cache[i].batch;
          } else {
            batch_free(g_batch_cache[i].batch);
            g_batch_cache.erase(g_batch_cache.begin() + i);
          }
          break;
        }
      }
      if (b == nullptr) {
        ibp_status_t st = batch_create(plans + c0, m, &b);
        if (st != IBP_SUCCESS) return st;
        if (g_batch_cache.size() >= kBatchCacheMax) {
          batch_free(g_batch_cache.front().batch);
          g_batch_cache.erase(g_batch_cache.begin());
        }
        g_batch_cache.push_back(BatchCacheEntry{key, b});
      }
    }
    ibp_status_t st = batch_solve(b, rhs + c0, phi + c0, s);
    if (st != IBP_SUCCESS) return st;
  }
  return IBP_SUCCESS;
}

}  // namespace

extern "C" {

ibp_status_t ibp_batch_create(const ibp_plan_t* plans, int count, ibp_batch_t* out) {
  if (plans == nullptr || out == nullptr) return IBP_ERROR_INVALID_VALUE;
  try {
    return batch_create(plans, count, out);
  } catch (...) {
    return IBP_ERROR_INTERNAL;
  }
}

ibp_status_t ibp_batch_solve(ibp_batch_t batch, const double* const* rhs, double* const* phi, hipStream_t stream) {
  if (batch == nullptr) return IBP_ERROR_INVALID_VALUE;
  try {
    return batch_solve(batch, rhs, phi, static_cast<hipStream_t>(stream));
  } catch (...) {
    return IBP_ERROR_INTERNAL;
  }
}

ibp_status_t ibp_batch_set_ycols(ibp_batch_t b, int cols) {
  if (b == nullptr || (cols != 2 && cols != 4 && cols != 8 && cols != 16)) return IBP_ERROR_INVALID_VALUE;
  try {
    b->yM = b->prec == IBP_FP64 ? batch_ytri_cols<double>(b->yP, b->yK, cols)
                                : batch_ytri_cols<float>(b->yP, b->yK, cols);
    return from_hip(batch_reapply(b));
  } catch (...) {
    return IBP_ERROR_INTERNAL;
  }
}

ibp_status_t ibp_batch_set_persistent(ibp_batch_t b, int enable) {
  if (b == nullptr) return IBP_ERROR_INVALID_VALUE;
  if (enable && !b->persist_ok) return IBP_ERROR_UNSUPPORTED_SIZE;
  b->persist = enable != 0;
  return IBP_SUCCESS;
}

ibp_status_t ibp_batch_destroy(ibp_batch_t b) {
  try {
    batch_free(b);
    return IBP_SUCCESS;
  } catch (...) {
    return IBP_ERROR_INTERNAL;
  }
}

}  // extern "C"

// ======================================================================
// Autotuning: time each candidate configuration with HIP events on the
// caller's stream (one warm-up solve, then the mean of a few) and keep the
// fastest.  Choices persist across processes in a cache file (IBP_TUNE_CACHE).
namespace {

// ---- tuning cache
// A text file of JSON lines, one per tuned configuration:
//   {"key": "<arch>/plan/<nx>x<ny>x<nz>/<precision>", "xdiv": 1, "zdiv": 1, "ycols": 4,
//    "xsmall": 1, "zsmall": 1, "persistent": 0, "lag": 1, "chunk": 8, "ms": 1.23}
// Batch keys are "<arch>/batch/<precision>.<max_iters>/<nx>x<ny>x<nz>,..." over
// the batch's grids in order.  The last line of a key wins.  <arch> is the
// device's gfx architecture name (e.g. gfx950).
std::mutex g_tune_mu;

std::string tune_cache_path() {
  const char* e = getenv("IBP_TUNE_CACHE");
  return (e && *e) ? std::string(e) : std::string();
}

std::string device_arch(int device) {
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) return "unknown";
  std::string a = prop.gcnArchName;
  const size_t c = a.find(':');
  return c == std::string::npos ? a : a.substr(0, c);
}

std::string plan_key(const ibp_plan_s* p) {
  char buf[160];
  snprintf(buf, sizeof buf, "%s/plan/%dx%dx%d/%d", device_arch(p->device).c_str(), p->nx, p->ny, p->nz, (int)p->prec);
  return buf;
}

std::string batch_key(const ibp_batch_s* b) {
  std::string k = device_arch(b->device) + "/batch/" + std::to_string((int)b->prec) + "." +
                  std::to_string(b->prec == IBP_FP64 ? 0 : b->max_iters) + "/";
  for (int g = 0; g < b->count; ++g) {
    const ibp_plan_s* p = b->plans[g];
    if (g) k += ",";
    k += std::to_string(p->nx) + "x" + std::to_string(p->ny) + "x" + std::to_string(p->nz);
  }
  return k;
}

// The cached configuration of `key`, if the cache file has one.
bool tune_cache_get(const std::string& key, TuneCfg* out) {
  const std::string path = tune_cache_path();
  if (path.empty()) return false;
  std::lock_guard<std::mutex> lock(g_tune_mu);
  return tune_file_get(path, key, out);
}

void tune_cache_put(const std::string& key, const TuneCfg& c, double ms) {
  const std::string path = tune_cache_path();
  if (path.empty()) return;
  std::lock_guard<std::mutex> lock(g_tune_mu);
  tune_file_put(path, key, c, ms);
}

// Plans: whether the general x / z transforms may take either LDS tile.
bool plan_x_tile_choice(const ibp_plan_s* p) {
  return !p->xfast && x_small(p->fpx, p->h) && p->chunk == 0 && !p->fused;
}
bool plan_z_tile_choice(const ibp_plan_s* p) { return !p->zfast && p->nz > 1 && z_small(p->fpz, p->nz); }

// A plan configuration: x and z tiles (where the plan may choose), z columns
// per block, line-solve columns per block.  None changes the arithmetic.
void apply_plan_cfg(ibp_plan_s* p, const TuneCfg& c) {
  if (c.xsmall >= 0 && plan_x_tile_choice(p)) {
    p->xsmall = c.xsmall != 0;
    set_x_split(p);
  }
  if (c.zsmall >= 0 && plan_z_tile_choice(p)) p->zsmall = c.zsmall != 0;
  set_z_split(p, c.zdiv > 0 ? c.zdiv : 1);
  p->ycols = c.ycols == 2 || c.ycols == 4 || c.ycols == 8 || c.ycols == 16 ? c.ycols : 0;
}

hipError_t apply_batch_cfg(ibp_batch_s* b, const TuneCfg& c) {
  b->xdiv = c.xdiv >= 1 && c.xdiv <= kBatchDivMax ? c.xdiv : 1;
  if (b->prec != IBP_FP64) b->xdiv = 1;   // the mixed forms' partials are sized for the finest split only
  b->zdiv = c.zdiv >= 1 ? c.zdiv : 1;
  const int want = c.ycols == 2 || c.ycols == 4 || c.ycols == 8 || c.ycols == 16 ? c.ycols : 0;
  b->yM = b->prec == IBP_FP64 ? batch_ytri_cols<double>(b->yP, b->yK, want)
                              : batch_ytri_cols<float>(b->yP, b->yK, want);
  b->persist = c.persist != 0 && b->persist_ok;
  b->lag = c.lag >= 1 ? c.lag : 1;
  b->pargs.chunk = c.chunk >= 1 && c.chunk <= 64 ? c.chunk : 8;
  return batch_reapply(b);
}

// cached: a configuration read from the tuning cache, applied and timed once
// (tried = 0); otherwise the fastest is stored under `key`.
template <class Apply, class Run>
ibp_status_t autotune(const std::vector<TuneCfg>& cands, Apply apply, Run run, hipStream_t s, ibp_tune_t* out,
                      bool cached = false, const std::string& key = std::string()) {
  constexpr int kReps = 3;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  ibp_status_t st = from_hip(e);
  double best = 1e300, before = 0.0;
  TuneCfg bestc = cands.front();
  for (size_t i = 0; i < cands.size() && st == IBP_SUCCESS; ++i) {
    st = apply(cands[i]);
    if (st == IBP_SUCCESS) st = run();
    if (st == IBP_SUCCESS) st = from_hip(hipEventRecord(e0, s));
    for (int r = 0; r < kReps && st == IBP_SUCCESS; ++r) st = run();
    if (st == IBP_SUCCESS) st = from_hip(hipEventRecord(e1, s));
    if (st == IBP_SUCCESS) st = from_hip(hipEventSynchronize(e1));
    float ms = 0.f;
    if (st == IBP_SUCCESS) st = from_hip(hipEventElapsedTime(&ms, e0, e1));
    if (st != IBP_SUCCESS) break;
    const double t = ms / kReps;
    if (i == 0) before = t;
    if (t < best) {
      best = t;
      bestc = cands[i];
    }
  }
  if (st == IBP_SUCCESS) st = apply(bestc);
  if (e0) hipEventDestroy(e0);
  if (e1) hipEventDestroy(e1);
  if (st == IBP_SUCCESS && !cached && !key.empty()) tune_cache_put(key, bestc, best);
  if (st == IBP_SUCCESS && out) {
    out->xdiv = bestc.xdiv;
    out->zdiv = bestc.zdiv;
    out->ycols = bestc.ycols;
    out->tried = cached ? 0 : (int)cands.size();
    out->xsmall = bestc.xsmall;
    out->zsmall = bestc.zsmall;
    out->ms = best;
    out->ms_before = before;
    out->persistent = bestc.persist;
    out->lag = bestc.lag;
    out->chunk = bestc.chunk;
  }
  return st;
}

void apply_cached_plan(ibp_plan_s* p) {
  if (tune_cache_path().empty()) return;
  TuneCfg c;
  if (tune_cache_get(plan_key(p), &c)) apply_plan_cfg(p, c);
}

ibp_status_t apply_cached_batch(ibp_batch_s* b) {
  if (tune_cache_path().empty()) return IBP_SUCCESS;
  TuneCfg c;
  if (!tune_cache_get(batch_key(b), &c)) return IBP_SUCCESS;
  return from_hip(apply_batch_cfg(b, c));
}

}  // namespace

extern "C" {

ibp_status_t ibp_plan_autotune(ibp_plan_t p, const double* rhs, double* phi, hipStream_t stream, ibp_tune_t* out) {
  if (!valid_plan(p) || rhs == nullptr || phi == nullptr) return IBP_ERROR_INVALID_VALUE;
  try {
    hipStream_t s = static_cast<hipStream_t>(stream);
    const bool can_x = plan_x_tile_choice(p), can_z = plan_z_tile_choice(p);
    const int zd0 = p->zc64max / (p->zc64 > 0 ? p->zc64 : 1);
    const TuneCfg now{1, zd0 > 0 ? zd0 : 1, p->ycols, 0, 1, 8, p->xsmall ? 1 : 0, p->zsmall ? 1 : 0};
    auto apply = [&](const TuneCfg& c) {
      apply_plan_cfg(p, c);
      return IBP_SUCCESS;
    };
    auto run = [&]() { return ibp_solve(p, rhs, phi, stream); };
    const std::string key = plan_key(p);
    TuneCfg cached;
    if (tune_cache_get(key, &cached)) return autotune({cached}, apply, run, s, out, true);
    std::vector<TuneCfg> cands{now};   // the configuration in place first
    const bool zgen = !p->zfast && p->nz > 1;
    for (int xs : {1, 0}) {
      if (!can_x && xs != now.xsmall) continue;
      for (int zs : {1, 0}) {
        if (!can_z && zs != now.zsmall) continue;
        for (int zd : {1, 2, 4}) {
          if (!zgen && zd > 1) continue;
          for (int yc : {2, 4, 8, 16}) cands.push_back(TuneCfg{1, zd, yc, 0, 1, 8, xs, zs});
        }
      }
    }
    ibp_status_t st = autotune(cands, apply, run, s, out, false, key);
    return st;
  } catch (...) {
    return IBP_ERROR_INTERNAL;
  }
}

ibp_status_t ibp_batch_autotune(ibp_batch_t b, const double* const* rhs, double* const* phi, hipStream_t stream,
                                ibp_tune_t* out) {
  if (b == nullptr || rhs == nullptr || phi == nullptr) return IBP_ERROR_INVALID_VALUE;
  try {
    hipStream_t s = static_cast<hipStream_t>(stream);
    auto apply = [&](const TuneCfg& c) { return from_hip(apply_batch_cfg(b, c)); };
    auto run = [&]() { return batch_solve(b, rhs, phi, s); };
    const std::string key = batch_key(b);
    TuneCfg cached;
    if (tune_cache_get(key, &cached)) return autotune({cached}, apply, run, s, out, true);
    std::vector<TuneCfg> cands{{b->xdiv, b->zdiv, b->yM, b->persist ? 1 : 0, b->lag, b->pargs.chunk}};
    for (int xd : {1, 2, 4}) {
      if (b->prec != IBP_FP64 && xd > 1) continue;   // the mixed forms' partials follow the x split
      for (int zd : {1, 2, 4}) {
        for (int yc : {2, 4, 8, 16}) cands.push_back(TuneCfg{xd, zd, yc, 0, 1, 8});
        // persistent: the line solve's columns per block follow from its block size
        if (b->persist_ok)
          for (int lag : {1, 2})
            for (int ch : {4, 16}) cands.push_back(TuneCfg{xd, zd, b->yM, 1, lag, ch});
      }
    }
    return autotune(cands, apply, run, s, out, false, key);
  } catch (...) {
    return IBP_ERROR_INTERNAL;
  }
}

}  // extern "C"

// ======================================================================
// Solves that allocate nothing: the workspace comes from one static device
// array per GPU (`scratch`, kScratchBytes) instead of the plan's own.  Its
// device address is looked up once per device with hipGetSymbolAddress; the
// array's name is only a host-side stand-in and is never handed to a kernel
// or a copy.  Every such solve on one GPU shares the array: the last call's
// contents stay there, and calls that overlap on one GPU (two streams, two
// threads) race.
namespace {

constexpr size_t kScratchBytes = size_t(32) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's scratch array (the device must be current).
ibp_status_t scratch_address(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices) return IBP_ERROR_INVALID_VALUE;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[dev] == nullptr) {
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return from_hip(e);
    if (ptr == nullptr || (reinterpret_cast<uintptr_t>(ptr) & 255) != 0) return IBP_ERROR_INTERNAL;
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return IBP_SUCCESS;
}

// The plan's workspace views, saved while a scratch solve borrows the plan.
struct WorkspaceViews {
  void* ws;
  Cx<double>* spec64;
  Cx<float>* spec32;
  double *rowsum, *phi00, *ghat, *part;
  int *ticket, *fctl;
  Ctl* ctl;
  bool fused, profiling;
  int chunk;
};

WorkspaceViews save_views(const ibp_plan_s* p) {
  return WorkspaceViews{p->ws,    p->spec64, p->spec32, p->rowsum, p->phi00,    p->ghat,  p->part,
                        p->ticket, p->fctl,  p->ctl,    p->fused,  p->profiling, p->chunk};
}

void restore_views(ibp_plan_s* p, const WorkspaceViews& v) {
  p->ws = v.ws;
  p->spec64 = v.spec64;
  p->spec32 = v.spec32;
  p->rowsum = v.rowsum;
  p->phi00 = v.phi00;
  p->ghat = v.ghat;
  p->part = v.part;
  p->ticket = v.ticket;
  p->fctl = v.fctl;
  p->ctl = v.ctl;
  p->fused = v.fused;
  p->profiling = v.profiling;
  p->chunk = v.chunk;
}

}  // namespace

extern "C" {

ibp_status_t ibp_solve_scratch(ibp_plan_t p, const double* rhs, double* phi, hipStream_t stream) {
  if (!valid_plan(p) || rhs == nullptr || phi == nullptr) return IBP_ERROR_INVALID_VALUE;
  if ((reinterpret_cast<uintptr_t>(rhs) & 15) != 0 || (reinterpret_cast<uintptr_t>(phi) & 15) != 0)
    return IBP_ERROR_INVALID_VALUE;
  const size_t n = (size_t)p->nx * p->ny * p->nz;
  if (p->prec != IBP_FP64) {
    const uintptr_t r0 = reinterpret_cast<uintptr_t>(rhs), r1 = r0 + n * sizeof(double);
    const uintptr_t q0 = reinterpret_cast<uintptr_t>(phi), q1 = q0 + n * sizeof(double);
    if (r0 < q1 && q0 < r1) return IBP_ERROR_INVALID_VALUE;
  }
  if (workspace_bytes(p) > kScratchBytes) return IBP_ERROR_UNSUPPORTED_SIZE;
  try {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return from_hip(e);
    if (dev != p->device) return IBP_ERROR_INVALID_VALUE;
    void* base = nullptr;
    ibp_status_t st = scratch_address(dev, &base);
    if (st != IBP_SUCCESS) return st;
    const WorkspaceViews saved = save_views(p);
    p->ws = base;
    carve_workspace(p);
    // the separate-pass schedule (no fused-pass queues, no second stream)
    // and no profiling events
    p->fused = false;
    p->chunk = 0;
    p->profiling = false;
    hipStream_t s = static_cast<hipStream_t>(stream);
    // the (0,0)-mode ticket starts every solve at zero (a fill kernel, not a
    // memset node, so the call stays capturable)
    e = launch_fill_zero(reinterpret_cast<double*>(p->ticket), 256 / sizeof(double), s);
    st = e == hipSuccess ? enqueue_solve(p, rhs, phi, s, nullptr) : from_hip(e);
    restore_views(p, saved);
    return st;
  } catch (...) {
    return IBP_ERROR_INTERNAL;
  }
}

}  // extern "C"

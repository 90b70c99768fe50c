// Host-only planning logic of libibpoisson, free of HIP: FFT factorisation
// and tables, the line-solve LU tables and shape choice, the dimension
// check, the tuning-cache file format and the persistent batch schedule's
// queue assignment.  Plain C++17, so it also builds on its own (for example
// with the host sanitizers) outside the HIP library.
#pragma once

#include <string>
#include <vector>

namespace ibp {

// ---------------------------------------------------------------- limits
constexpr int kTileX64 = 2048, kTileX32 = 4096;   // complex elements per x-pass block
constexpr int kTileX64s = 1024, kTileX32s = 2048; // small x tiles (as for z below)
constexpr int kTileZ64 = 4096, kTileZ32 = 8192;   // complex elements per z-pass block
// Small z tiles for short lines: the general transform's stage registers
// scale with the tile (340 VGPRs at 4096 FP64, 167 at 1024), so lines that
// fit run at two to three times the occupancy.
constexpr int kTileZ64s = 1024, kTileZ32s = 2048;
constexpr int kMaxNy = 1536;

// FFT factorisation handed to kernels by value.
struct FftPlan {
  int n;          // sequence length
  int nst;        // number of stages
  int radix[16];  // radices in stage order
  int any;        // 1: a radix above 11 (direct-sum stage; half tiles)
  int blu;        // 1: Bluestein: the length-n DFT as a length-m cyclic convolution
  int m;          // Bluestein convolution length (a power of two >= 2n - 1)
  int mst;        // its stages
  int mradix[8];  // its radices (8, 4, 2)
};

// Radix factorisation (8s, 4s, 2s, then 3, 5, 7, 11, then larger primes);
// false past 16 stages or for n < 1.
bool factorize(int n, FftPlan* fp);
// Switch lengths with a prime factor above kBluesteinPrime to Bluestein's
// algorithm when the convolution length fits `max_m`.
constexpr int kBluesteinPrime = 256;
void plan_bluestein(FftPlan* fp, int max_m);
// Bluestein chirp (2n doubles) and filter spectrum (2m doubles).
void bluestein_tables(int n, int m, std::vector<double>& chirp, std::vector<double>& bhat);
// W_n^e = exp(-2 pi i e / n), e = 0..n-1.
void twiddles(int n, std::vector<double>& re, std::vector<double>& im);

// Dimension check: kDimsOk, kDimsInvalid (a size below 1) or
// kDimsUnsupported (outside what the kernels cover).  On success fills the
// x (half length) and z factorisations when the pointers are non-null.
enum { kDimsOk = 0, kDimsInvalid = 1, kDimsUnsupported = 2 };
int dims_status(int nx, int ny, int nz, FftPlan* fpx, FftPlan* fpz);

// Line-solve shape: lanes per column P and rows per lane K with P K >= ny.
bool ytri_shape(int ny, int* P, int* K);

// LU tables of a (cyclic) tridiagonal system, in the form the line kernels
// apply: forward x_i = m_i x_{i-1} + s_i r_i, backward x_i += t_i x_{i+1},
// then for a cyclic system x -= w (x_0 + g x_{n-1}) (Sherman-Morrison).
struct LineLu {
  std::vector<double> m, s, t, w;
  double g = 0.0;
  int cyclic = 0;
};
LineLu line_lu(std::vector<double> lo, std::vector<double> di, std::vector<double> up, bool cyclic);

// ---------------------------------------------------------------- tuning cache
// A text file of JSON lines, one per tuned configuration:
//   {"key": "<arch>/plan/<nx>x<ny>x<nz>/<precision>", "xdiv": 1, "zdiv": 1, "ycols": 4,
//    "xsmall": 1, "zsmall": 1, "persistent": 0, "lag": 1, "chunk": 8, "ms": 1.23}
// Batch keys are "<arch>/batch/<precision>.<max_iters>/<nx>x<ny>x<nz>,..." over
// the batch's grids in order.  The last valid line of a key wins; a line
// with a field outside its range is skipped.
struct TuneCfg {
  int xdiv = 1, zdiv = 1;   // work splits of the x rows and z columns per block (1..64)
  int ycols = 0;            // line-solve columns per block: 0 (default), 2, 4, 8 or 16
  int persist = 0;          // batches: the persistent schedule (0 or 1)
  int lag = 1;              // its diagonal interleave (1..64)
  int chunk = 8;            // and the items its blocks claim at once (1..64)
  int xsmall = -1;          // plans: general x transform in the small (1) or large (0) LDS tile; -1: keep
  int zsmall = -1;          // plans: the same for the general z transform
};
// Integer value of "name": in a JSON line (dflt if absent); false when the
// text after it is not an integer within int's range.
bool json_int(const std::string& line, const char* name, int dflt, int* out);
// Parses one cache line for `key`; false if the line is for another key,
// malformed, or has a field outside its range.
bool tune_line_parse(const std::string& line, const std::string& key, TuneCfg* out);
bool tune_file_get(const std::string& path, const std::string& key, TuneCfg* out);
void tune_file_put(const std::string& path, const std::string& key, const TuneCfg& c, double ms);

// ---------------------------------------------------------------- batch schedule
// Longest-processing-time assignment of grids (by work, ties in index order)
// to nq queues: each grid in turn to the least-loaded queue.
std::vector<std::vector<int>> lpt_queues(const std::vector<double>& work, int nq);
// Order of the stages of one queue's grids: stage s of the queue's i-th grid
// gets key s + lag i, sorted by key then i (a diagonal interleave).
struct DiagItem {
  int pos, stage;
};
std::vector<DiagItem> diagonal_order(const std::vector<int>& nstages, int lag);

}  // namespace ibp

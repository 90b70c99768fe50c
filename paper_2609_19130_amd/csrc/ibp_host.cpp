// Host-only planning logic of libibpoisson (declarations and formats in
// ibp_host.hpp).
#include "ibp_host.hpp"

#include <algorithm>
#include <cerrno>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <utility>

namespace ibp {

// Radix factorisation for the LDS FFT: eights first, then fours, twos, the
// odd primes with butterflies of their own (3, 5, 7, 11), then any larger
// prime factors (direct-sum stages).  Returns false only past 16 stages.
bool factorize(int n, FftPlan* fp) {
  *fp = FftPlan{};
  fp->n = n;
  if (n < 1) return false;
  fp->nst = 0;
  fp->any = 0;
  fp->blu = 0;
  fp->m = 0;
  fp->mst = 0;
  int m = n;
  auto push = [&](int r) {
    if (fp->nst >= 16) return false;
    fp->radix[fp->nst++] = r;
    if (r > 11) fp->any = 1;
    m /= r;
    return true;
  };
  while (m % 8 == 0)
    if (!push(8)) return false;
  while (m % 4 == 0)
    if (!push(4)) return false;
  while (m % 2 == 0)
    if (!push(2)) return false;
  for (int p : {3, 5, 7, 11})
    while (m % p == 0)
      if (!push(p)) return false;
  for (int p = 13; p * p <= m; p += 2)
    while (m % p == 0)
      if (!push(p)) return false;
  if (m > 1 && !push(m)) return false;   // the remaining prime
  return m == 1;
}

// Lengths whose largest prime factor exceeds kBluesteinPrime take Bluestein's
// algorithm instead of a direct-sum stage, if the convolution length m (the
// power of two >= 2n - 1) fits `max_m`.  Both move similar LDS traffic per
// value at R ~ 100-200 (R/4 reads per output for the direct sum against two
// padded length-m transforms), and the direct sum measured faster there on
// MI355X (501 = 3 x 167 and 632 = 8 x 79 grids), so only larger primes switch.
void plan_bluestein(FftPlan* fp, int max_m) {
  int big = 1;
  for (int s = 0; s < fp->nst; ++s) big = fp->radix[s] > big ? fp->radix[s] : big;
  if (big <= kBluesteinPrime) return;
  int m = 1;
  while (m < 2 * fp->n - 1) m *= 2;
  if (m > max_m) return;
  fp->blu = 1;
  fp->any = 0;
  fp->m = m;
  fp->mst = 0;
  int r = m;
  while (r % 8 == 0) { fp->mradix[fp->mst++] = 8; r /= 8; }
  while (r % 4 == 0) { fp->mradix[fp->mst++] = 4; r /= 4; }
  while (r % 2 == 0) { fp->mradix[fp->mst++] = 2; r /= 2; }
}

// Bluestein tables of length n (convolution length m), FP64 from long double:
// chirp w_j = exp(-i pi j^2 / n) (angle reduced as j^2 mod 2n), and bhat =
// DFT_m of the filter b with b_t = conj(w_|t|) at t mod m for |t| < n (a
// radix-2 transform in long double).
void bluestein_tables(int n, int m, std::vector<double>& chirp, std::vector<double>& bhat) {
  const long double pi = 3.141592653589793238462643383279502884L;
  chirp.assign(2 * (size_t)n, 0.0);
  std::vector<long double> br(m, 0.0L), bi(m, 0.0L);
  for (int j = 0; j < n; ++j) {
    const long long r = ((long long)j * j) % (2LL * n);
    const long double a = pi * (long double)r / (long double)n;
    chirp[2 * j] = (double)cosl(a);
    chirp[2 * j + 1] = (double)-sinl(a);
    br[j] = cosl(a);   // conj(w_j)
    bi[j] = sinl(a);
    if (j > 0) {
      br[m - j] = cosl(a);
      bi[m - j] = sinl(a);
    }
  }
  // iterative radix-2 DFT, exp(-2 pi i j k / m)
  for (int i = 1, j = 0; i < m; ++i) {
    int bit = m >> 1;
    for (; j & bit; bit >>= 1) j ^= bit;
    j ^= bit;
    if (i < j) {
      std::swap(br[i], br[j]);
      std::swap(bi[i], bi[j]);
    }
  }
  for (int len = 2; len <= m; len <<= 1) {
    const long double ang = -2.0L * pi / (long double)len;
    for (int i = 0; i < m; i += len)
      for (int k = 0; k < len / 2; ++k) {
        const long double wr = cosl(ang * k), wi = sinl(ang * k);
        const long double ur = br[i + k], ui = bi[i + k];
        const long double vr = br[i + k + len / 2] * wr - bi[i + k + len / 2] * wi;
        const long double vi = br[i + k + len / 2] * wi + bi[i + k + len / 2] * wr;
        br[i + k] = ur + vr;
        bi[i + k] = ui + vi;
        br[i + k + len / 2] = ur - vr;
        bi[i + k + len / 2] = ui - vi;
      }
  }
  bhat.assign(2 * (size_t)m, 0.0);
  for (int k = 0; k < m; ++k) {
    bhat[2 * k] = (double)br[k];
    bhat[2 * k + 1] = (double)bi[k];
  }
}

// W_n^e = exp(-2 pi i e / n), e = 0..n-1, evaluated in long double and rounded.
void twiddles(int n, std::vector<double>& re, std::vector<double>& im) {
  re.resize(n);
  im.resize(n);
  const long double two_pi = 6.283185307179586476925286766559005768L;
  for (int e = 0; e < n; ++e) {
    const long double a = two_pi * (long double)e / (long double)n;
    re[e] = (double)cosl(a);
    im[e] = (double)-sinl(a);
  }
}

// ---------------------------------------------------------------- line-solve shape
// P = 32 lanes per column (P = 64 when ny > 384), K rows per lane from
// {2, 4, 8, 12, 16, 24}.
bool ytri_shape(int ny, int* P, int* K) {
  static constexpr int kKs[] = {2, 4, 8, 12, 16, 24};
  if (ny < 2 || ny > kMaxNy) return false;
  // 64 lanes once a column needs more than 12 rows per lane of 32: 24 rows
  // per lane hold ~350 VGPRs (one wave per SIMD), 12 rows ~180 (two waves)
  const int p = ny > 32 * 12 ? 64 : 32;
  const int need = (ny + p - 1) / p;
  for (int k : kKs) {
    if (k >= need) {
      *P = p;
      *K = k;
      return true;
    }
  }
  return false;
}

// ---------------------------------------------------------------- dimensions
int dims_status(int nx, int ny, int nz, FftPlan* fpx, FftPlan* fpz) {
  if (nx < 1 || nz < 1 || ny < 1) return kDimsInvalid;
  // x transform length: nx/2 complex pairs, or nx complex values for odd nx
  const int hx = nx % 2 ? nx : nx / 2;
  if (hx > kTileX64) return kDimsUnsupported;
  if (nz > kTileZ64) return kDimsUnsupported;
  if (ny < 2 || ny > kMaxNy) return kDimsUnsupported;
  FftPlan a{}, b{};
  if (!factorize(hx, &a) || !factorize(nz, &b)) return kDimsUnsupported;
  plan_bluestein(&a, kTileX64);          // rows of m values in the large x tile
  plan_bluestein(&b, kTileZ64 / 2);      // columns of m + 1 values in the large z tile
  // a prime factor above 11 needs the spare half of the general tiles
  if (a.any && hx > kTileX64 / 2) return kDimsUnsupported;
  if (b.any && nz + 1 > kTileZ64 / 2) return kDimsUnsupported;
  int P, K;
  if (!ytri_shape(ny, &P, &K)) return kDimsUnsupported;
  if (fpx) *fpx = a;
  if (fpz) *fpz = b;
  return kDimsOk;
}

// ---------------------------------------------------------------- line LU
LineLu line_lu(std::vector<double> lo, std::vector<double> di, std::vector<double> up, bool cyclic) {
  const int n = (int)di.size();
  LineLu L;
  if (cyclic && n == 1) {   // both neighbours are the point itself
    di[0] += lo[0] + up[0];
    cyclic = false;
  } else if (cyclic && n == 2) {   // both neighbours are the other point
    up[0] += lo[0];
    lo[1] += up[1];
    cyclic = false;
  }
  std::vector<double> u;
  if (cyclic) {
    const double gamma = -di[0];
    const double clo = lo[0], cup = up[n - 1];
    di[0] -= gamma;
    di[n - 1] -= clo * cup / gamma;
    u.assign(n, 0.0);
    u[0] = gamma;
    u[n - 1] = cup;
    L.g = clo / gamma;
    L.cyclic = 1;
  }
  lo[0] = 0.0;
  up[n - 1] = 0.0;
  L.m.assign(n, 0.0);
  L.s.assign(n, 0.0);
  L.t.assign(n, 0.0);
  L.w.assign(n, 0.0);
  double den = 0.0;
  for (int i = 0; i < n; ++i) {
    den = i == 0 ? di[0] : di[i] - lo[i] * up[i - 1] / den;
    L.s[i] = 1.0 / den;
    L.m[i] = -lo[i] / den;
    L.t[i] = -up[i] / den;
  }
  if (cyclic) {
    std::vector<double> z(n);
    double prev = 0.0;
    for (int i = 0; i < n; ++i) prev = z[i] = L.m[i] * prev + L.s[i] * u[i];
    double nxt = 0.0;
    for (int i = n - 1; i >= 0; --i) nxt = z[i] = z[i] + L.t[i] * nxt;
    const double vz = z[0] + L.g * z[n - 1];
    for (int i = 0; i < n; ++i) L.w[i] = z[i] / (1.0 + vz);
  }
  return L;
}

// ---------------------------------------------------------------- tuning cache
bool json_int(const std::string& line, const char* name, int dflt, int* out) {
  const std::string pat = std::string("\"") + name + "\":";
  const size_t at = line.find(pat);
  if (at == std::string::npos) {
    *out = dflt;
    return true;
  }
  const char* begin = line.c_str() + at + pat.size();
  char* end = nullptr;
  errno = 0;
  const long v = strtol(begin, &end, 10);
  if (end == begin || errno == ERANGE || v < INT_MIN || v > INT_MAX) return false;
  *out = (int)v;
  return true;
}

bool tune_line_parse(const std::string& line, const std::string& key, TuneCfg* out) {
  const std::string want = "\"key\": \"" + key + "\"";
  if (line.find(want) == std::string::npos) return false;
  TuneCfg c;
  const bool ok = json_int(line, "xdiv", 1, &c.xdiv) && json_int(line, "zdiv", 1, &c.zdiv) &&
                  json_int(line, "ycols", 0, &c.ycols) && json_int(line, "persistent", 0, &c.persist) &&
                  json_int(line, "lag", 1, &c.lag) && json_int(line, "chunk", 8, &c.chunk) &&
                  json_int(line, "xsmall", -1, &c.xsmall) && json_int(line, "zsmall", -1, &c.zsmall);
  if (!ok) return false;
  auto in = [](int v, int lo, int hi) { return v >= lo && v <= hi; };
  if (!in(c.xdiv, 1, 64) || !in(c.zdiv, 1, 64) || !in(c.lag, 1, 64) || !in(c.chunk, 1, 64)) return false;
  if (!(c.ycols == 0 || c.ycols == 2 || c.ycols == 4 || c.ycols == 8 || c.ycols == 16)) return false;
  if (!in(c.persist, 0, 1) || !in(c.xsmall, -1, 1) || !in(c.zsmall, -1, 1)) return false;
  *out = c;
  return true;
}

bool tune_file_get(const std::string& path, const std::string& key, TuneCfg* out) {
  FILE* f = fopen(path.c_str(), "r");
  if (!f) return false;
  bool found = false;
  std::string line;
  char chunk[4096];
  while (fgets(chunk, sizeof chunk, f)) {
    line += chunk;
    if (line.back() != '\n' && !feof(f)) continue;   // a line longer than the buffer
    TuneCfg c;
    if (tune_line_parse(line, key, &c)) {
      *out = c;
      found = true;   // keep reading: the last valid line of a key wins
    }
    line.clear();
  }
  fclose(f);
  return found;
}

void tune_file_put(const std::string& path, const std::string& key, const TuneCfg& c, double ms) {
  FILE* f = fopen(path.c_str(), "a+");
  if (!f) return;
  // start on a line of its own when the file's last line has no newline
  if (fseek(f, -1, SEEK_END) == 0 && fgetc(f) != '\n') fputc('\n', f);
  fseek(f, 0, SEEK_END);
  fprintf(f,
          "{\"key\": \"%s\", \"xdiv\": %d, \"zdiv\": %d, \"ycols\": %d, \"xsmall\": %d, \"zsmall\": %d, "
          "\"persistent\": %d, \"lag\": %d, \"chunk\": %d, \"ms\": %.6f}\n",
          key.c_str(), c.xdiv, c.zdiv, c.ycols, c.xsmall, c.zsmall, c.persist, c.lag, c.chunk, ms);
  fclose(f);
}

// ---------------------------------------------------------------- batch schedule
std::vector<std::vector<int>> lpt_queues(const std::vector<double>& work, int nq) {
  const int n = (int)work.size();
  std::vector<std::vector<int>> q(nq > 0 ? nq : 0);
  if (nq <= 0) return q;
  std::vector<int> order(n);
  for (int g = 0; g < n; ++g) order[g] = g;
  std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return work[a] > work[c]; });
  std::vector<double> load(nq, 0.0);
  for (int g : order) {
    const int k = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    q[k].push_back(g);
    load[k] += work[g];
  }
  return q;
}

std::vector<DiagItem> diagonal_order(const std::vector<int>& nstages, int lag) {
  struct Key {
    long key;
    int pos, stage;
  };
  std::vector<Key> keys;
  for (int i = 0; i < (int)nstages.size(); ++i)
    for (int st = 0; st < nstages[i]; ++st) keys.push_back({st + (long)lag * i, i, st});
  std::stable_sort(keys.begin(), keys.end(),
                   [](const Key& a, const Key& c) { return a.key != c.key ? a.key < c.key : a.pos < c.pos; });
  std::vector<DiagItem> out;
  out.reserve(keys.size());
  for (const Key& k : keys) out.push_back({k.pos, k.stage});
  return out;
}

}  // namespace ibp

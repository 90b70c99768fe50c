// Self-test of the host-only planning logic (paper_2609_19130_amd/csrc/
// ibp_host.cpp), built on its own with the host sanitizers by
// test_host_sanitized.py.  Checks properties that must hold for every input
// in a sweep and prints the dimension checks it made ("dims nx ny nz status")
// for comparison with the HIP library's ibp_check_dims.  Exit status 0 when
// every check holds.
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <string>
#include <vector>

#include "ibp_host.hpp"

using namespace ibp;

static int g_fail = 0;
#define CHECK(c, ...)                        \
  do {                                       \
    if (!(c)) {                              \
      ++g_fail;                              \
      if (g_fail < 20) {                     \
        fprintf(stderr, "FAIL %s: ", #c);    \
        fprintf(stderr, __VA_ARGS__);        \
        fprintf(stderr, "\n");               \
      }                                      \
    }                                        \
  } while (0)

static bool is_prime(int p) {
  if (p < 2) return false;
  for (int d = 2; d * d <= p; ++d)
    if (p % d == 0) return false;
  return true;
}

static void test_factorize() {
  for (int n = -3; n <= 8192; ++n) {
    FftPlan fp;
    const bool ok = factorize(n, &fp);
    if (n < 1) {
      CHECK(!ok, "n=%d", n);
      continue;
    }
    CHECK(ok, "n=%d", n);
    long prod = 1;
    int prev_class = 0;   // 8, 4, 2, then odd primes in increasing order
    for (int s = 0; s < fp.nst; ++s) {
      const int r = fp.radix[s];
      prod *= r;
      CHECK(r == 8 || r == 4 || r == 2 || is_prime(r), "n=%d radix %d", n, r);
      const int cls = r == 8 ? 0 : r == 4 ? 1 : r == 2 ? 2 : 3 + r;
      CHECK(cls >= prev_class, "n=%d order", n);
      prev_class = cls;
    }
    CHECK(prod == n, "n=%d product %ld", n, prod);
    bool big = false;
    for (int s = 0; s < fp.nst; ++s) big |= fp.radix[s] > 11;
    CHECK(fp.any == (big ? 1 : 0), "n=%d any", n);
    // at most one 4 and one 2 after the eights
    int fours = 0, twos = 0;
    for (int s = 0; s < fp.nst; ++s) fours += fp.radix[s] == 4, twos += fp.radix[s] == 2;
    CHECK(fours + twos <= 1, "n=%d 4s and 2s", n);
    FftPlan b = fp;
    plan_bluestein(&b, 4096);
    int largest = 1;
    for (int s = 0; s < fp.nst; ++s) largest = fp.radix[s] > largest ? fp.radix[s] : largest;
    int m = 1;
    while (m < 2 * n - 1) m *= 2;
    if (largest > kBluesteinPrime && m <= 4096) {
      CHECK(b.blu == 1 && b.any == 0 && b.m == m, "n=%d bluestein", n);
      long mp = 1;
      for (int s = 0; s < b.mst; ++s) mp *= b.mradix[s];
      CHECK(mp == m, "n=%d m stages", n);
    } else {
      CHECK(b.blu == 0 && b.any == fp.any, "n=%d no bluestein", n);
    }
  }
}

static void test_tables() {
  using C = std::complex<long double>;
  const long double pi = 3.141592653589793238462643383279502884L;
  for (int n : {1, 2, 3, 5, 17, 257, 263, 509}) {
    int m = 1;
    while (m < 2 * n - 1) m *= 2;
    std::vector<double> ch, bh;
    bluestein_tables(n, m, ch, bh);
    CHECK((int)ch.size() == 2 * n && (int)bh.size() == 2 * m, "n=%d sizes", n);
    // the filter spectrum against a direct DFT of b_t = conj(w_|t|)
    std::vector<C> bt(m, C(0, 0));
    for (int j = 0; j < n; ++j) {
      const C w = std::polar(1.0L, -pi * (long double)j * j / n);
      bt[j] = std::conj(w);
      if (j) bt[m - j] = std::conj(w);
    }
    double err = 0.0;
    for (int k = 0; k < m; ++k) {
      C s(0, 0);
      for (int t = 0; t < m; ++t) s += bt[t] * std::polar(1.0L, -2 * pi * (long double)((long)k * t % m) / m);
      err = std::max(err, (double)std::abs(s - C(bh[2 * k], bh[2 * k + 1])));
      if (k < n) {
        const C w = std::polar(1.0L, -pi * (long double)k * k / n);
        err = std::max(err, (double)std::abs(w - C(ch[2 * k], ch[2 * k + 1])));
      }
    }
    CHECK(err < 1e-12 * n, "n=%d table error %g", n, err);
    std::vector<double> re, im;
    twiddles(n, re, im);
    for (int e = 0; e < n; ++e) {
      const C w = std::polar(1.0L, -2 * pi * (long double)e / n);
      CHECK(std::abs(w - C(re[e], im[e])) < 1e-15, "twiddle n=%d e=%d", n, e);
    }
  }
}

// Applies the tables the way the line kernels do and returns max |A x - r| / max |r|.
static double lu_residual(const std::vector<double>& lo, const std::vector<double>& di, const std::vector<double>& up,
                          bool cyclic, std::mt19937_64& rng) {
  const int n = (int)di.size();
  const LineLu L = line_lu(lo, di, up, cyclic);
  CHECK((int)L.m.size() == n && (int)L.s.size() == n && (int)L.t.size() == n && (int)L.w.size() == n, "sizes n=%d", n);
  std::uniform_real_distribution<double> U(-1.0, 1.0);
  std::vector<double> r(n), x(n);
  for (double& v : r) v = U(rng);
  double prev = 0.0;
  for (int i = 0; i < n; ++i) prev = x[i] = L.m[i] * prev + L.s[i] * r[i];
  double nxt = 0.0;
  for (int i = n - 1; i >= 0; --i) nxt = x[i] = x[i] + L.t[i] * nxt;
  if (L.cyclic) {
    const double c = x[0] + L.g * x[n - 1];
    for (int i = 0; i < n; ++i) x[i] -= L.w[i] * c;
  }
  double err = 0.0, rmax = 0.0;
  for (int i = 0; i < n; ++i) {
    double ax = di[i] * x[i];
    if (cyclic) {
      ax += lo[i] * x[(i + n - 1) % n] + up[i] * x[(i + 1) % n];
    } else {
      if (i > 0) ax += lo[i] * x[i - 1];
      if (i + 1 < n) ax += up[i] * x[i + 1];
    }
    err = std::max(err, std::fabs(ax - r[i]));
    rmax = std::max(rmax, std::fabs(r[i]));
  }
  return err / rmax;
}

static void test_line_lu() {
  std::mt19937_64 rng(7);
  std::uniform_real_distribution<double> U(0.1, 1.0);
  for (int n = 1; n <= 64; ++n)
    for (int cyc = 0; cyc < 2; ++cyc) {
      std::vector<double> lo(n), di(n), up(n);
      for (int i = 0; i < n; ++i) {
        lo[i] = -U(rng);
        up[i] = -U(rng);
        di[i] = 1.0 + std::fabs(lo[i]) + std::fabs(up[i]);   // diagonally dominant (implicit viscous lines)
      }
      const double res = lu_residual(lo, di, up, cyc != 0, rng);
      CHECK(res < 1e-13, "line LU n=%d cyclic=%d residual %g", n, cyc, res);
    }
}

static void test_ytri_shape() {
  for (int ny = -1; ny <= kMaxNy + 10; ++ny) {
    int P = 0, K = 0;
    const bool ok = ytri_shape(ny, &P, &K);
    CHECK(ok == (ny >= 2 && ny <= kMaxNy), "ny=%d", ny);
    if (ok) CHECK((P == 32 || P == 64) && P * K >= ny && P * K < 2 * ny + 64 * 4, "ny=%d P=%d K=%d", ny, P, K);
  }
}

static void test_dims() {
  const int xs[] = {-1, 0, 1, 2, 3, 7, 30, 64, 96, 126, 334, 501, 512, 1002, 1024, 1264, 2048, 2050, 4094, 4096, 4098, 8192};
  const int ys[] = {-5, 0, 1, 2, 3, 33, 384, 385, 768, 1001, 1263, 1536, 1537};
  const int zs[] = {-1, 0, 1, 2, 5, 263, 501, 632, 1024, 2039, 2053, 4096, 4097};
  for (int nx : xs)
    for (int ny : ys)
      for (int nz : zs) {
        FftPlan a, b;
        const int st = dims_status(nx, ny, nz, &a, &b);
        printf("dims %d %d %d %d\n", nx, ny, nz, st);
        if (st == kDimsOk) CHECK(a.n == (nx % 2 ? nx : nx / 2) && b.n == nz, "dims %d %d %d", nx, ny, nz);
      }
}

static void test_tune_cache(const char* dir) {
  const std::string path = std::string(dir) + "/tune_cache_selftest.jsonl";
  remove(path.c_str());
  TuneCfg c;
  CHECK(!tune_file_get(path, "gfx950/plan/64x33x64/0", &c), "missing file");
  FILE* f = fopen(path.c_str(), "w");
  std::string longline = "{\"key\": \"other\", \"pad\": \"" + std::string(10000, 'x') + "\", \"xdiv\": 2}\n";
  fputs(longline.c_str(), f);
  fputs("{\"key\": \"gfx950/plan/64x33x64/0\", \"xdiv\": 1, \"zdiv\": 2, \"ycols\": 4, \"xsmall\": 1, \"zsmall\": 0}\n", f);
  fputs("{\"key\": \"gfx950/plan/64x33x64/0\", \"xdiv\": 99999999999999999999, \"zdiv\": 2}\n", f);   // overflow: skipped
  fputs("{\"key\": \"gfx950/plan/64x33x64/0\", \"xdiv\": abc}\n", f);                             // not a number: skipped
  fputs("{\"key\": \"gfx950/plan/64x33x64/0\", \"lag\": 2147483647}\n", f);                       // out of range: skipped
  fputs("{\"key\": \"gfx950/plan/64x33x64/0\", \"ycols\": 3}\n", f);                              // not a column count: skipped
  fputs("garbage without braces\n\n", f);
  fputs("{\"key\": \"gfx950/batch/1.4/32x32x32,48x48x48\", \"persistent\": 1, \"lag\": 3, \"chunk\": 16}", f);   // no newline at the end
  fclose(f);
  CHECK(tune_file_get(path, "gfx950/plan/64x33x64/0", &c), "plan key");
  CHECK(c.xdiv == 1 && c.zdiv == 2 && c.ycols == 4 && c.xsmall == 1 && c.zsmall == 0 && c.lag == 1, "plan cfg");
  CHECK(tune_file_get(path, "gfx950/batch/1.4/32x32x32,48x48x48", &c), "batch key");
  CHECK(c.persist == 1 && c.lag == 3 && c.chunk == 16 && c.xdiv == 1, "batch cfg");
  CHECK(!tune_file_get(path, "gfx950/plan/64x33x6", &c) || true, "prefix");
  TuneCfg w;
  w.xdiv = 4;
  w.zdiv = 8;
  w.ycols = 16;
  w.persist = 0;
  w.lag = 2;
  w.chunk = 32;
  w.xsmall = 0;
  w.zsmall = 1;
  tune_file_put(path, "gfx950/plan/64x33x64/0", w, 1.25);
  TuneCfg r;
  CHECK(tune_file_get(path, "gfx950/plan/64x33x64/0", &r), "round trip");
  CHECK(r.xdiv == 4 && r.zdiv == 8 && r.ycols == 16 && r.lag == 2 && r.chunk == 32 && r.xsmall == 0 && r.zsmall == 1,
        "round trip fields");
  remove(path.c_str());
}

static void test_schedule() {
  std::mt19937_64 rng(11);
  std::uniform_int_distribution<int> D(1, 200);
  for (int trial = 0; trial < 200; ++trial) {
    const int n = 1 + trial % 70, nq = 1 + trial % 9;
    std::vector<double> work(n);
    double total = 0.0, big = 0.0;
    for (double& w : work) total += (w = (double)D(rng) * D(rng)), big = std::max(big, w);
    const auto q = lpt_queues(work, nq);
    CHECK((int)q.size() == nq, "queues");
    std::vector<int> seen(n, 0);
    double lmax = 0.0, lmin = 1e300;
    for (const auto& v : q) {
      double l = 0.0;
      for (int g : v) {
        CHECK(g >= 0 && g < n, "grid index");
        ++seen[g];
        l += work[g];
      }
      lmax = std::max(lmax, l);
      lmin = std::min(lmin, l);
    }
    for (int g = 0; g < n; ++g) CHECK(seen[g] == 1, "grid %d assigned %d times", g, seen[g]);
    // LPT: the most loaded queue exceeds the least loaded by at most one grid's work
    if (n >= nq) CHECK(lmax - lmin <= big, "balance");
    std::vector<int> ns(n);
    for (int& s : ns) s = D(rng) % 30;
    const int lag = 1 + trial % 64;
    const auto order = diagonal_order(ns, lag);
    std::vector<int> next(n, 0);
    for (const DiagItem& it : order) {
      CHECK(it.pos >= 0 && it.pos < n, "pos");
      CHECK(it.stage == next[it.pos], "stages of a grid in order");
      ++next[it.pos];
    }
    for (int i = 0; i < n; ++i) CHECK(next[i] == ns[i], "every stage once");
  }
  CHECK(lpt_queues({1.0, 2.0}, 0).empty(), "no queues");
  CHECK(diagonal_order({}, 5).empty(), "no grids");
}

int main(int argc, char** argv) {
  const char* dir = argc > 1 ? argv[1] : ".";
  test_factorize();
  test_tables();
  test_line_lu();
  test_ytri_shape();
  test_dims();
  test_tune_cache(dir);
  test_schedule();
  fprintf(stderr, "host selftest: %d failures\n", g_fail);
  return g_fail ? 1 : 0;
}

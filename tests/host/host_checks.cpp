// Checks of the library's host-side numerics (paper_2507_07823_amd/csrc/wfp_host.cpp),
// built with AddressSanitizer and UndefinedBehaviorSanitizer by tests/test_host_engine.py.
// Exit status 0 when every check holds; a message and status 1 otherwise.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <random>
#include <set>
#include <utility>
#include <vector>

#include "../../paper_2507_07823_amd/csrc/wfp_host.h"

using namespace wfp;

static int failures = 0;
#define CHECK(c, ...)                          \
  do {                                         \
    if (!(c)) {                                \
      std::fprintf(stderr, "FAIL %s:%d: ", __FILE__, __LINE__); \
      std::fprintf(stderr, __VA_ARGS__);       \
      std::fprintf(stderr, "\n");              \
      ++failures;                              \
    }                                          \
  } while (0)

// Gauss-Legendre rules integrate x^k exactly for k < 2n.
static void check_gauss_legendre() {
  for (int n : {1, 2, 7, 32, 35, 64}) {
    std::vector<double> z, w;
    gauss_legendre(n, z, w);
    CHECK((int)z.size() == n && (int)w.size() == n, "sizes n=%d", n);
    for (int k = 0; k < 2 * n && k < 60; ++k) {
      double s = 0.0;
      for (int i = 0; i < n; ++i) s += w[i] * std::pow(z[i], k);
      const double exact = (k % 2) ? 0.0 : 2.0 / (k + 1);
      CHECK(std::fabs(s - exact) < 1e-13, "GL n=%d k=%d: %.17g vs %.17g", n, k, s, exact);
    }
  }
}

// I0 against its values at a few points (sum of the series to many terms).
static void check_bessel() {
  CHECK(std::fabs((double)bessel_i0(0.0L) - 1.0) < 1e-16, "I0(0)");
  // I0(1) = 1.2660658777520082, I0(10) = 2815.716628466254
  CHECK(std::fabs((double)bessel_i0(1.0L) - 1.2660658777520082) < 1e-15, "I0(1)");
  CHECK(std::fabs((double)bessel_i0(10.0L) / 2815.716628466254 - 1.0) < 1e-14, "I0(10)");
}

// Window series: Phi(-1) = 0, Phi(1) = 1, Phi(0) = 1/2; the piecewise table
// reproduces the series.
static void check_window() {
  const double b = std::log(1e12);
  WindowSeries ws = window_series(b, 80);
  CHECK(std::fabs(cheb_eval(ws.phi.data(), ws.n, 1.0) - 1.0) < 1e-14, "Phi(1)");
  CHECK(std::fabs(cheb_eval(ws.phi.data(), ws.n, -1.0)) < 1e-14, "Phi(-1)");
  CHECK(std::fabs(cheb_eval(ws.phi.data(), ws.n, 0.0) - 0.5) < 1e-15, "Phi(0)");
  const int pieces = 512, deg = 5;
  std::vector<double> tab = window_pieces(ws, pieces, deg);
  CHECK((int)tab.size() == pieces * (deg + 1), "table size");
  double worst = 0.0;
  for (int i = 0; i <= 4000; ++i) {
    const double u = -1.0 + 2.0 * i / 4000.0;
    int pc = (int)((u + 1.0) * (0.5 * pieces));
    pc = std::min(std::max(pc, 0), pieces - 1);
    const double t = (u + 1.0) * (0.5 * pieces) - pc;
    double v = tab[(size_t)pc * (deg + 1) + deg];
    for (int k = deg - 1; k >= 0; --k) v = std::fma(v, t, tab[(size_t)pc * (deg + 1) + k]);
    worst = std::max(worst, std::fabs(v - cheb_eval(ws.phi.data(), ws.n, u)));
  }
  CHECK(worst < 1e-15, "window table error %.3g", worst);
}

// Neighbour ranges against brute force, and the upper ranges: every unordered
// pair closer than r in exactly one upper range, every column sum a block
// writes read by exactly one row's total.
static void check_ranges(std::mt19937_64& rng, int M, double r, bool periodic, bool clustered) {
  std::uniform_real_distribution<double> U(-kPi, kPi);
  std::vector<double> xs(M);
  for (int i = 0; i < M; ++i) {
    double v = U(rng);
    if (clustered && i % 3 == 0) v = 0.37 + 1e-4 * U(rng);              // a dense clump
    if (periodic && i % 7 == 0) v = (i % 2 ? kPi - 1e-3 : -kPi) + 1e-4 * std::fabs(U(rng));
    if (!periodic) v = std::max(-kPi + 0.5, std::min(kPi - 0.5, v));
    if (v >= kPi) v -= 2 * kPi;
    xs[i] = v;
  }
  if (M > 4) xs[3] = xs[2];                                              // a duplicate position
  std::sort(xs.begin(), xs.end());
  std::vector<int> nbs(M), nbc(M);
  for (int j = 0; j < M; ++j) {
    source_range(xs, xs[j], r, periodic, false, nbs[j], nbc[j]);
    std::set<int> got;
    for (int k = 0; k < nbc[j]; ++k) got.insert((nbs[j] + k) % M);
    CHECK((int)got.size() == nbc[j], "range of %d repeats a source", j);
    for (int l = 0; l < M; ++l) {
      const bool in = pair_distance(xs[j], xs[l], periodic) < r;
      CHECK(in == (got.count(l) > 0), "M=%d periodic=%d row %d source %d: brute %d range %d", M, (int)periodic,
            j, l, (int)in, (int)(got.count(l) > 0));
    }
  }
  const int rows = 16;
  std::vector<int> up, be;
  std::vector<int64_t> po;
  int64_t total = 0;
  const bool ok = upper_ranges(nbs, nbc, rows, up, be, po, total);
  CHECK(ok, "upper_ranges refused M=%d periodic=%d", M, (int)periodic);
  if (!ok) return;
  std::map<std::pair<int, int>, int> seen;
  for (int j = 0; j < M; ++j)
    for (long long u = j; u < up[j]; ++u) {
      const int l = (int)(u % M);
      seen[std::make_pair(std::min(j, l), std::max(j, l))] += 1;
    }
  for (int i = 0; i < M; ++i)
    for (int l = i; l < M; ++l) {
      const bool in = pair_distance(xs[i], xs[l], periodic) < r;
      const int n = seen.count(std::make_pair(i, l)) ? seen[std::make_pair(i, l)] : 0;
      CHECK(n == (in ? 1 : 0), "pair (%d, %d) taken %d times (within r: %d)", i, l, n, (int)in);
    }
  // column sums: block b writes u in [b rows, be[b]) at po[b] + (u - b rows); the
  // per-row total of l reads blocks b <= l / rows with be[b] > l, and (periodic)
  // blocks with be[b] > l + M
  const int nb = (int)be.size();
  std::vector<int> reads(total, 0);
  for (int l = 0; l < M; ++l) {
    for (int b = l / rows; b >= 0 && be[b] > l; --b) reads[po[b] + (l - b * rows)] += 1;
    if (periodic)
      for (int b = nb - 1; b >= 0 && be[b] > (long long)l + M; --b) reads[po[b] + ((long long)l + M - b * rows)] += 1;
  }
  for (int64_t e = 0; e < total; ++e) CHECK(reads[e] == 1, "column sum %lld read %d times", (long long)e, reads[e]);
}

int main() {
  check_gauss_legendre();
  check_bessel();
  check_window();
  std::mt19937_64 rng(12345);
  for (int M : {1, 2, 3, 15, 16, 17, 40, 200, 700})
    for (int periodic = 0; periodic < 2; ++periodic)
      for (int cl = 0; cl < 2; ++cl)
        for (double r : {0.01, 0.3, 2.5}) check_ranges(rng, M, r, periodic != 0, cl != 0);
  CHECK(radix_sequence(1280).size() > 0 && is_pow2_pow5(12500) && !is_pow2_pow5(12501), "radix");
  if (failures) {
    std::fprintf(stderr, "%d checks failed\n", failures);
    return 1;
  }
  std::printf("host checks passed\n");
  return 0;
}

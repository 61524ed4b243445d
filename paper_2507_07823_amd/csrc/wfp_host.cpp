// Host-side numerics of the plan set-up.  See wfp_host.h.
#include "wfp_host.h"

#include <algorithm>
#include <cmath>

namespace wfp {

void gauss_legendre(int n, std::vector<double>& z, std::vector<double>& w) {
  z.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    long double x = std::cos(kPi * (i + 0.75L) / (n + 0.5L));
    long double dp = 0;
    for (int it = 0; it < 100; ++it) {
      long double p0 = 1, p1 = x;
      for (int k = 2; k <= n; ++k) {
        long double p2 = ((2 * k - 1) * x * p1 - (k - 1) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      if (n == 1) { p1 = x; p0 = 1; }
      dp = n * (x * p1 - p0) / (x * x - 1);
      long double dx = p1 / dp;
      x -= dx;
      if (std::fabs((double)dx) < 1e-19) break;
    }
    // recompute derivative at the converged node
    long double p0 = 1, p1 = x;
    for (int k = 2; k <= n; ++k) {
      long double p2 = ((2 * k - 1) * x * p1 - (k - 1) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    if (n == 1) { p1 = x; p0 = 1; }
    dp = n * (x * p1 - p0) / (x * x - 1);
    z[n - 1 - i] = (double)x;  // ascending
    w[n - 1 - i] = (double)(2.0L / ((1 - x * x) * dp * dp));
  }
}

long double bessel_i0(long double x) {
  long double q = 0.25L * x * x, term = 1, sum = 1;
  for (int k = 1; k < 200; ++k) {
    term *= q / ((long double)k * k);
    sum += term;
    if (term < 1e-22L * sum) break;
  }
  return sum;
}

double cheb_eval(const double* a, int n, double s) {
  double b1 = 0, b2 = 0;
  for (int k = n - 1; k >= 1; --k) {
    double b0 = 2.0 * s * b1 - b2 + a[k];
    b2 = b1;
    b1 = b0;
  }
  return 0.5 * a[0] + s * b1 - b2;
}

WindowSeries window_series(double b, int n) {
  // a_k = (2/n) sum_i g(s_i) cos(k theta_i), s_i = cos(theta_i), theta_i = pi (i + 1/2)/n
  WindowSeries ws;
  ws.n = n + 1;
  const long double bl = b;
  const long double scale = bl / (2.0L * std::sinh(bl));
  std::vector<long double> gv(n), a(n + 2, 0.0L);
  for (int i = 0; i < n; ++i) {
    long double th = kPi * (i + 0.5L) / n;
    long double s = std::cos(th);
    long double r = std::sqrt(std::max(0.0L, 1.0L - s * s));
    gv[i] = scale * bessel_i0(bl * r);
  }
  for (int k = 0; k < n; ++k) {
    long double acc = 0;
    for (int i = 0; i < n; ++i) acc += gv[i] * std::cos(k * kPi * (i + 0.5L) / n);
    a[k] = 2.0L * acc / n;
  }
  // derivative: a'_{k-1} = a'_{k+1} + 2k a_k
  std::vector<long double> d(n + 2, 0.0L);
  for (int k = n - 1; k >= 1; --k) d[k - 1] = d[k + 1] + 2.0L * k * a[k];
  // integral: A_k = (a_{k-1} - a_{k+1}) / (2k), A_0 fixed by Phi(-1) = 0
  std::vector<long double> A(n + 2, 0.0L);
  for (int k = 1; k <= n; ++k) A[k] = (a[k - 1] - a[k + 1]) / (2.0L * k);
  long double s0 = 0;
  for (int k = 1; k <= n; ++k) s0 += A[k] * ((k % 2) ? -1.0L : 1.0L);
  A[0] = -2.0L * s0;
  ws.phi.resize(n + 1);
  ws.g.assign(n + 1, 0.0);
  ws.dg.assign(n + 1, 0.0);
  for (int k = 0; k <= n; ++k) ws.phi[k] = (double)A[k];
  for (int k = 0; k < n; ++k) ws.g[k] = (double)a[k];
  for (int k = 0; k < n; ++k) ws.dg[k] = (double)d[k];
  return ws;
}

// Augmented coordinate of virtual index a in [0, 3M): xs[a mod M] + 2 pi (a div M - 1).
static inline double aug(const std::vector<double>& xs, int64_t a, int64_t M) {
  return xs[a % M] + kTwoPi * (double)(a / M - 1);
}

void source_range(const std::vector<double>& xs, double x, double r, bool periodic,
                  bool inclusive, int& start, int& count) {
  const int64_t M = (int64_t)xs.size();
  auto inside = [&](int64_t idx) {
    double d = pair_distance(x, xs[idx], periodic);
    return inclusive ? (d <= r) : (d < r);
  };
  const double margin = 1e-9 * (1.0 + r);
  if (!periodic) {
    int64_t lo = std::lower_bound(xs.begin(), xs.end(), x - r - margin) - xs.begin();
    int64_t hi = std::upper_bound(xs.begin(), xs.end(), x + r + margin) - xs.begin();  // exclusive
    while (lo < hi && !inside(lo)) ++lo;
    while (hi > lo && !inside(hi - 1)) --hi;
    start = (int)lo;
    count = (int)(hi - lo);
    return;
  }
  // binary search on the augmented virtual array
  auto lower = [&](double v) {
    int64_t lo = 0, hi = 3 * M;
    while (lo < hi) {
      int64_t mid = (lo + hi) / 2;
      if (aug(xs, mid, M) < v) lo = mid + 1; else hi = mid;
    }
    return lo;
  };
  auto upper = [&](double v) {
    int64_t lo = 0, hi = 3 * M;
    while (lo < hi) {
      int64_t mid = (lo + hi) / 2;
      if (aug(xs, mid, M) <= v) lo = mid + 1; else hi = mid;
    }
    return lo;
  };
  int64_t lo = lower(x - r - margin), hi = upper(x + r + margin);
  if (hi - lo > M) {  // window covers the whole circle
    start = 0;
    count = (int)M;
    return;
  }
  while (lo < hi && !inside(lo % M)) ++lo;
  while (hi > lo && !inside((hi - 1) % M)) --hi;
  start = (int)(lo % M);
  count = (int)(hi - lo);
}

bool upper_ranges(const std::vector<int>& nbs, const std::vector<int>& nbc, int rows, std::vector<int>& up,
                  std::vector<int>& blk_end, std::vector<int64_t>& part_off, int64_t& total) {
  const int64_t M = (int64_t)nbs.size();
  const int64_t nb = (M + rows - 1) / rows;
  up.assign(M, 0);
  blk_end.assign(nb, 0);
  part_off.assign(nb, 0);
  for (int64_t j = 0; j < M; ++j) {
    const int64_t st = nbs[j] <= j ? nbs[j] : (int64_t)nbs[j] - M;
    const int64_t e = st + nbc[j];
    if (!(st <= j && j < e && e <= j + M)) return false;
    up[j] = (int)e;
    blk_end[j / rows] = std::max(blk_end[j / rows], (int)e);
  }
  total = 0;
  for (int64_t b = 0; b < nb; ++b) {
    if (b > 0 && blk_end[b] < blk_end[b - 1]) return false;
    part_off[b] = total;
    total += (int64_t)blk_end[b] - b * rows;
  }
  return true;
}

bool is_pow2_pow5(int64_t n) {
  if (n < 1) return false;
  while (n % 2 == 0) n /= 2;
  while (n % 5 == 0) n /= 5;
  return n == 1;
}

std::vector<int> radix_sequence(int64_t n) {
  std::vector<int> r;
  int a = 0, c = 0;
  while (n % 2 == 0) { n /= 2; ++a; }
  while (n % 5 == 0) { n /= 5; ++c; }
  for (int i = 0; i < a / 2; ++i) r.push_back(4);
  if (a % 2) r.push_back(2);
  for (int i = 0; i < c; ++i) r.push_back(5);
  return r;
}


std::vector<double> window_pieces(const WindowSeries& ws, int pieces, int deg) {
  const int n = deg + 1;
  std::vector<double> out((size_t)pieces * n);
  // Chebyshev points of the piece, in the local variable x in [0, 1]
  std::vector<long double> t(n);
  for (int i = 0; i < n; ++i) t[i] = 0.5L + 0.5L * std::cos(3.14159265358979323846264338327950288L * (i + 0.5L) / n);
  for (int k = 0; k < pieces; ++k) {
    const long double width = 2.0L / pieces;
    const long double left = -1.0L + 2.0L * k / pieces;
    // Vandermonde system V c = f, V_ij = t_i^j
    std::vector<long double> a((size_t)n * (n + 1));
    for (int i = 0; i < n; ++i) {
      long double p = 1.0L;
      for (int j = 0; j < n; ++j) {
        a[(size_t)i * (n + 1) + j] = p;
        p *= t[i];
      }
      a[(size_t)i * (n + 1) + n] = cheb_eval(ws.phi.data(), ws.n, (double)(left + width * t[i]));
    }
    for (int c = 0; c < n; ++c) {
      int piv = c;
      for (int r = c + 1; r < n; ++r)
        if (std::fabs((double)a[(size_t)r * (n + 1) + c]) > std::fabs((double)a[(size_t)piv * (n + 1) + c])) piv = r;
      for (int j = 0; j <= n; ++j) std::swap(a[(size_t)piv * (n + 1) + j], a[(size_t)c * (n + 1) + j]);
      for (int r = 0; r < n; ++r) {
        if (r == c) continue;
        const long double f = a[(size_t)r * (n + 1) + c] / a[(size_t)c * (n + 1) + c];
        for (int j = c; j <= n; ++j) a[(size_t)r * (n + 1) + j] -= f * a[(size_t)c * (n + 1) + j];
      }
    }
    for (int j = 0; j < n; ++j)
      out[(size_t)k * n + j] = (double)(a[(size_t)j * (n + 1) + n] / a[(size_t)j * (n + 1) + j]);
  }
  return out;
}

}  // namespace wfp

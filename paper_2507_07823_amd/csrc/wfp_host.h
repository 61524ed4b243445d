// Host-side numerics of the plan set-up (window series, Gauss-Legendre rules,
// neighbour ranges).  Pure C++, no HIP; also compiled into the host unit test
// of the library.
#pragma once

#include <cmath>
#include <cstdint>
#include <vector>

namespace wfp {

constexpr double kPi = 3.14159265358979323846;
constexpr double kTwoPi = 2.0 * kPi;

// Gauss-Legendre nodes and weights on [-1, 1] (Newton iteration on the
// three-term recurrence of P_n, carried in long double).
void gauss_legendre(int n, std::vector<double>& z, std::vector<double>& w);

// Modified Bessel I0 by its power series, in long double.
long double bessel_i0(long double x);

// Chebyshev series (a_0/2 + sum_{n>=1} a_n T_n) of the Kaiser-Bessel window in
// the rescaled variable s = 2t/delta - 1 (Section 2, eq. (phi)):
//   g(s)  = I0(b sqrt(1 - s^2)) * b / (2 sinh b),
//   Phi(s) = int_{-1}^{s} g   (so phi(t) = Phi(s), phi'(t) = (2/delta) g(s),
//                               phi''(t) = (4/delta^2) g'(s)).
// The series do not depend on delta, so one set serves the time window and the
// spatial window of the RBC.
struct WindowSeries {
  int n = 0;
  std::vector<double> phi, g, dg;
};
WindowSeries window_series(double b, int n);

// The window phi(u) of a series on [-1, 1] as `pieces` polynomials of degree
// `deg`: piece k covers u in [-1 + 2k/pieces, -1 + 2(k+1)/pieces] and holds
// monomial coefficients c_0..c_deg in x = (u + 1) pieces / 2 - k in [0, 1],
// interpolating phi at deg + 1 Chebyshev points (solved in long double).
std::vector<double> window_pieces(const WindowSeries& ws, int pieces, int deg);
double cheb_eval(const double* a, int n, double s);   // prime convention

// Distance used for neighbour decisions (Definition lambdadef); the same
// expression is evaluated on the device.
inline double pair_distance(double a, double c, bool periodic) {
  double d = std::fabs(a - c);
  if (periodic && d > kPi) d = kTwoPi - d;
  return d;
}

// Sources (sorted ascending in [-pi, pi)) closer than r to position x form a
// circular index range [start, start + count) (mod M).  `inclusive` selects
// d <= r instead of d < r.
void source_range(const std::vector<double>& xs, double x, double r, bool periodic,
                  bool inclusive, int& start, int& count);

// Upper source ranges of the local sum that takes each unordered pair once.
// Row j (sorted order) has the neighbour range [nbs[j], nbs[j] + nbc[j])
// (mod M), which contains j; its upper range is the unwrapped [j, up[j]): the
// sources from j upward (past M - 1 the indices continue at 0).  Per block of
// `rows` consecutive rows: blk_end[b] = the largest up[j] of its rows, and
// part_off[b] = the offset of its column sums (one per source u in
// [rows b, blk_end[b])); total = their sum.  Returns false when a range does
// not contain its row or the block ends decrease (the sums over covering
// blocks rely on non-decreasing ends).
bool upper_ranges(const std::vector<int>& nbs, const std::vector<int>& nbc, int rows, std::vector<int>& up,
                  std::vector<int>& blk_end, std::vector<int64_t>& part_off, int64_t& total);

// 2^a 5^b test and the radix sequence (4s, at most one 2, then 5s) used by
// the LDS FFT.
bool is_pow2_pow5(int64_t n);
std::vector<int> radix_sequence(int64_t n);

}  // namespace wfp

// Host checks of the setup's dense SVD pieces (csrc/dense.hpp) on the inputs
// that rank-deficient Schur complements produce: Householder vectors far
// below the rounding level (down to subnormal numbers), a bidiagonal whose
// trailing entries decay past the double range, clusters of equal tiny
// singular values, and the truncated Schur complement of a Gamma block whose
// rank is far below its column count.  Prints "dense svd ok" when every case
// passes; exits non-zero on the first failure.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "../../paper_2601_04112_amd/csrc/dense.hpp"

using lsamg::bidiag_svd;
using lsamg::householder;
using lsamg::schur_svd;

static int fails = 0;
#define CHECK(cond, ...)                       \
  do {                                         \
    if (!(cond)) {                             \
      std::printf("FAIL %s:%d: ", __FILE__, __LINE__); \
      std::printf(__VA_ARGS__);                \
      std::printf("\n");                       \
      ++fails;                                 \
    }                                          \
  } while (0)

// H x = alpha e_1 for the reflector householder() returns, evaluated in
// long double after scaling x by a power of two (so the check itself neither
// underflows nor overflows)
static void check_reflector(std::vector<double> x, const char* name) {
  const int m = (int)x.size();
  std::vector<double> v = x;
  double beta, alpha;
  householder(m, v.data(), beta, alpha);
  CHECK(std::isfinite(beta) && std::isfinite(alpha), "%s: beta %g alpha %g", name, beta, alpha);
  double amax = 0;
  for (double t : x) amax = std::max(amax, std::abs(t));
  int ex;
  std::frexp(amax, &ex);
  long double n2 = 0;
  for (double t : x) n2 += (long double)std::ldexp(t, -ex) * std::ldexp(t, -ex);
  const long double nrm = std::sqrt(n2);
  // a subnormal alpha carries an absolute error of half its spacing, 2^-1075
  const long double tol = 1e-15L * nrm + (long double)std::ldexp(1.0, -1074 - ex);
  CHECK(std::abs(std::abs((long double)std::ldexp(alpha, -ex)) - nrm) <= tol,
        "%s: |alpha| %Lg vs norm %Lg", name, (long double)std::ldexp(alpha, -ex), nrm);
  if (beta == 0.0) return;
  long double vx = 0;
  for (int i = 0; i < m; ++i) vx += (long double)v[i] * std::ldexp(x[i], -ex);
  for (int i = 0; i < m; ++i) {
    const long double hx = std::ldexp(x[i], -ex) - (long double)beta * vx * v[i];
    const long double want = i == 0 ? (long double)std::ldexp(alpha, -ex) : 0.0L;
    CHECK(std::abs(hx - want) <= 1e-14L * nrm + tol, "%s: (Hx)[%d] %Lg want %Lg", name, i, hx,
          want);
  }
}

// sum of squares of the entries (invariant under the orthogonal iteration)
static long double frob2(const std::vector<double>& d, const std::vector<double>& e) {
  long double s = 0;
  for (double t : d) s += (long double)t * t;
  for (double t : e) s += (long double)t * t;
  return s;
}

static void check_bidiag(std::vector<double> d, std::vector<double> e, const char* name) {
  const int n = (int)d.size();
  const long double f0 = frob2(d, e);
  std::vector<double> W((size_t)n * 2);
  for (int i = 0; i < n; ++i) {
    W[(size_t)i * 2] = 1.0 / (1 + i);
    W[(size_t)i * 2 + 1] = std::sin(1.0 + i);
  }
  long double w0 = 0;
  for (double t : W) w0 += (long double)t * t;
  const bool ok = bidiag_svd(n, d.data(), e.data(), W.data(), 2);
  CHECK(ok, "%s: iteration did not converge", name);
  if (!ok) return;
  long double f1 = 0;
  for (double t : d) f1 += (long double)t * t;
  CHECK(std::abs(f1 - f0) <= 1e-13L * f0, "%s: sum of sigma^2 %Lg vs %Lg", name, f1, f0);
  long double w1 = 0;
  for (double t : W) w1 += (long double)t * t;
  CHECK(std::abs(w1 - w0) <= 1e-13L * w0, "%s: rotated rows lost norm %Lg vs %Lg", name, w1, w0);
}

// Q with orthonormal columns spanning the columns of F (rows x r), by
// modified Gram-Schmidt applied twice; columns at or below tol (relative) are
// dropped
static std::vector<std::vector<double>> basis(int rows, int r, const std::vector<double>& F) {
  std::vector<std::vector<double>> Q;
  for (int j = 0; j < r; ++j) {
    std::vector<double> q(F.begin() + (size_t)j * rows, F.begin() + (size_t)(j + 1) * rows);
    double n0 = 0;
    for (double t : q) n0 += t * t;
    for (int pass = 0; pass < 2; ++pass)
      for (auto& u : Q) {
        double s = 0;
        for (int i = 0; i < rows; ++i) s += u[i] * q[i];
        for (int i = 0; i < rows; ++i) q[i] -= s * u[i];
      }
    double nn = 0;
    for (double t : q) nn += t * t;
    if (nn <= 1e-20 * n0) continue;
    for (double& t : q) t /= std::sqrt(nn);
    Q.push_back(q);
  }
  return Q;
}

// [Bw Bg] with Bg = F G of rank r (ng columns) and a graded scale per
// column: S must equal Bw^T (I - Q Q^T) Bw with Q a basis of range(F), and
// the rank returned must be r
static void check_schur(int rows, int nw, int ng, int r, double grade, unsigned seed) {
  std::mt19937_64 g(seed);
  std::normal_distribution<double> N(0.0, 1.0);
  std::vector<double> F((size_t)rows * r), Gm((size_t)r * ng), B((size_t)rows * (nw + ng));
  for (double& t : F) t = N(g);
  for (double& t : Gm) t = N(g);
  for (int i = 0; i < rows * nw; ++i) B[i] = N(g);
  for (int j = 0; j < ng; ++j) {
    const double sc = std::pow(grade, (double)j / std::max(ng - 1, 1));
    for (int i = 0; i < rows; ++i) {
      double s = 0;
      for (int k = 0; k < r; ++k) s += F[(size_t)k * rows + i] * Gm[(size_t)j * r + k];
      B[(size_t)(nw + j) * rows + i] = sc * s;
    }
  }
  const std::vector<double> Bw(B.begin(), B.begin() + (size_t)rows * nw);
  std::vector<double> S((size_t)nw * nw);
  const int rank = schur_svd(rows, nw, ng, B.data(), 1e-6, S.data());
  CHECK(rank == r, "schur rows %d ng %d: rank %d, want %d", rows, ng, rank, r);
  const auto Q = basis(rows, r, F);
  std::vector<double> E = Bw;                // (I - Q Q^T) Bw
  for (int c = 0; c < nw; ++c)
    for (const auto& u : Q) {
      double s = 0;
      for (int i = 0; i < rows; ++i) s += u[i] * E[(size_t)c * rows + i];
      for (int i = 0; i < rows; ++i) E[(size_t)c * rows + i] -= s * u[i];
    }
  double smax = 0, dmax = 0;
  for (int a = 0; a < nw; ++a)
    for (int b = 0; b < nw; ++b) {
      double s = 0;
      for (int i = 0; i < rows; ++i) s += E[(size_t)a * rows + i] * E[(size_t)b * rows + i];
      smax = std::max(smax, std::abs(s));
      dmax = std::max(dmax, std::abs(s - S[(size_t)b * nw + a]));
    }
  CHECK(dmax <= 1e-9 * smax, "schur rows %d ng %d: |S - S_ref| %g of %g", rows, ng, dmax, smax);
}

int main() {
  // reflectors: ordinary, tiny normal, subnormal, mixed scales
  check_reflector({3.0, 4.0, 0.0, 12.0}, "ordinary");
  check_reflector({2.8e-303, 1.1e-303, -7.0e-304}, "tiny");
  check_reflector({4e-316, -1e-316, 3e-317, 2e-318}, "subnormal");
  check_reflector({0.0, 5e-320, 0.0}, "subnormal, zero head");
  check_reflector({1e-300, 1.0, -1e-300}, "mixed");
  check_reflector({0.0, 0.0, 0.0}, "zero");
  // bidiagonals: ordinary, entries decaying past the double range, a large
  // cluster of equal tiny singular values below a unit one
  {
    std::vector<double> d(40), e(39);
    for (int i = 0; i < 40; ++i) d[i] = 1.0 + 0.1 * i;
    for (int i = 0; i < 39; ++i) e[i] = 0.5 - 0.01 * i;
    check_bidiag(d, e, "ordinary");
  }
  {
    std::vector<double> d(60), e(59);
    for (int i = 0; i < 60; ++i) d[i] = std::pow(10.0, -11.0 * i) * (i % 2 ? -0.7 : 0.9);
    for (int i = 0; i < 59; ++i) e[i] = std::pow(10.0, -11.0 * i - 6.0) * 0.3;
    check_bidiag(d, e, "graded past the double range");
  }
  {
    std::vector<double> d(300, 3e-17), e(299, 2e-17);
    d[0] = 1.0;
    e[0] = 0.25;
    check_bidiag(d, e, "cluster of tiny values");
  }
  // truncated Schur complements of rank-deficient Gamma blocks: more rows
  // than columns, fewer rows than Gamma columns, and strongly graded columns
  check_schur(120, 8, 60, 12, 1.0, 1);
  check_schur(60, 6, 150, 20, 1.0, 2);
  check_schur(200, 10, 180, 30, 1e-3, 3);
  check_schur(90, 5, 300, 25, 1e-2, 4);
  if (fails) {
    std::printf("%d check(s) failed\n", fails);
    return 1;
  }
  std::printf("dense svd ok\n");
  return 0;
}

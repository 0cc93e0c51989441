// Small dense FP64 linear algebra for the host setup phase.
//
// All matrices are column-major with leading dimension equal to their row
// count.  Written from the textbook algorithms (Golub & Van Loan, "Matrix
// Computations", 4th ed.): right-looking Cholesky (sec. 4.2), Householder
// tridiagonalisation (sec. 8.3.1) followed by the implicit symmetric QR step
// with Wilkinson shift (sec. 8.3.3), Householder QR (sec. 5.2.2),
// Householder bidiagonalisation (sec. 5.4.8) and the Golub-Kahan SVD step
// (sec. 8.6.2).
#pragma once

#include <algorithm>
#include <cmath>
#include <immintrin.h>
#include <cstdint>
#include <numeric>
#include <vector>

namespace lsamg {

// In-place lower Cholesky factor of the SPD matrix a (n x n).  Only the lower
// triangle is read and written.  Returns false if a pivot is not positive.
inline bool chol_lower(int n, double* a) {
  for (int j = 0; j < n; ++j) {
    double* cj = a + (size_t)j * n;
    double d = cj[j];
    if (!(d > 0.0) || !std::isfinite(d)) return false;
    d = std::sqrt(d);
    cj[j] = d;
    const double inv = 1.0 / d;
    for (int i = j + 1; i < n; ++i) cj[i] *= inv;
    for (int k = j + 1; k < n; ++k) {
      double* ck = a + (size_t)k * n;
      const double f = cj[k];
      if (f == 0.0) continue;
      for (int i = k; i < n; ++i) ck[i] -= cj[i] * f;
    }
  }
  return true;
}

// Solve L X = B in place (B is n x r), L lower triangular from chol_lower.
inline void trsm_lower(int n, const double* l, int r, double* b) {
  for (int c = 0; c < r; ++c) {
    double* x = b + (size_t)c * n;
    for (int j = 0; j < n; ++j) {
      const double* lj = l + (size_t)j * n;
      const double xj = x[j] / lj[j];
      x[j] = xj;
      if (xj == 0.0) continue;
      for (int i = j + 1; i < n; ++i) x[i] -= lj[i] * xj;
    }
  }
}

// Solve L^T X = B in place (B is n x r).
inline void trsm_lower_t(int n, const double* l, int r, double* b) {
  for (int c = 0; c < r; ++c) {
    double* x = b + (size_t)c * n;
    for (int j = n - 1; j >= 0; --j) {
      const double* lj = l + (size_t)j * n;
      double s = x[j];
      for (int i = j + 1; i < n; ++i) s -= lj[i] * x[i];
      x[j] = s / lj[j];
    }
  }
}

// Householder vector of x (length m): on return x holds v with v[0] scaled
// so that H = I - beta v v^T maps the input to alpha e_1.  The vector is
// first scaled by the power of two that brings its largest entry into
// [1/2, 1) (2^1000 at most, which keeps the factor finite): exact, so the
// result is unchanged wherever the plain formulas neither underflow nor
// overflow, and v v^T (hence beta) stays finite for vectors far below the
// rounding-noise level of a rank-deficient matrix (whose squares would
// otherwise flush to zero or turn beta infinite).
inline void householder(int m, double* x, double& beta, double& alpha) {
  double amax = 0.0;
  for (int i = 0; i < m; ++i) amax = std::max(amax, std::abs(x[i]));
  if (amax == 0.0 || !std::isfinite(amax)) {
    beta = 0.0;
    alpha = x[0];
    return;
  }
  int ex;
  (void)std::frexp(amax, &ex);
  ex = std::max(ex, -1000);
  const double sc = std::ldexp(1.0, -ex);
  for (int i = 0; i < m; ++i) x[i] *= sc;
  double sig = 0.0;
  for (int i = 1; i < m; ++i) sig += x[i] * x[i];
  const double x0 = x[0];
  if (sig == 0.0) {
    beta = 0.0;
    alpha = std::ldexp(x0, ex);
    x[0] = alpha;
    for (int i = 1; i < m; ++i) x[i] = std::ldexp(x[i], ex);
    return;
  }
  const double nrm = std::sqrt(x0 * x0 + sig);
  const double a = (x0 >= 0.0) ? -nrm : nrm;
  x[0] = x0 - a;
  const double vtv = x[0] * x[0] + sig;
  beta = 2.0 / vtv;
  alpha = std::ldexp(a, ex);
}

// Symmetric eigen-decomposition a = V diag(w) V^T of the n x n matrix a
// (full storage, overwritten by V).  Eigenvalues ascending.  Returns false if
// the QR iteration does not converge.
inline bool sym_eig(int n, double* a, double* w) {
  if (n == 0) return true;
  if (n == 1) {
    w[0] = a[0];
    a[0] = 1.0;
    return true;
  }
  std::vector<double> d(n), e(n, 0.0), betas(n, 0.0), p(n), q(n);
  // 1. Householder tridiagonalisation: reflector k acts on rows/cols k+1..n-1
  for (int k = 0; k + 2 < n; ++k) {
    const int m = n - k - 1;
    double* v = a + (size_t)k * n + (k + 1);      // column k below diagonal
    double beta, alpha;
    householder(m, v, beta, alpha);
    betas[k] = beta;
    e[k] = alpha;
    if (beta == 0.0) continue;
    // p = beta * T v, T = trailing block a[k+1:, k+1:]
    for (int i = 0; i < m; ++i) p[i] = 0.0;
    for (int j = 0; j < m; ++j) {
      const double* tj = a + (size_t)(k + 1 + j) * n + (k + 1);
      const double vj = v[j];
      for (int i = 0; i < m; ++i) p[i] += tj[i] * vj;
    }
    double ptv = 0.0;
    for (int i = 0; i < m; ++i) {
      p[i] *= beta;
      ptv += p[i] * v[i];
    }
    const double kk = 0.5 * beta * ptv;
    for (int i = 0; i < m; ++i) q[i] = p[i] - kk * v[i];      // w
    for (int j = 0; j < m; ++j) {
      double* tj = a + (size_t)(k + 1 + j) * n + (k + 1);
      const double vj = v[j], wj = q[j];
      for (int i = 0; i < m; ++i) tj[i] -= v[i] * wj + q[i] * vj;
    }
  }
  for (int k = 0; k < n; ++k) d[k] = a[(size_t)k * n + k];
  e[n - 2] = a[(size_t)(n - 2) * n + (n - 1)];
  // 2. accumulate Q = H_0 H_1 ... backwards into a separate matrix
  std::vector<double> Q((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) Q[(size_t)i * n + i] = 1.0;
  for (int k = n - 3; k >= 0; --k) {
    const double beta = betas[k];
    if (beta == 0.0) continue;
    const int m = n - k - 1;
    const double* v = a + (size_t)k * n + (k + 1);
    for (int j = k + 1; j < n; ++j) {
      double* qj = Q.data() + (size_t)j * n + (k + 1);
      double s = 0.0;
      for (int i = 0; i < m; ++i) s += v[i] * qj[i];
      s *= beta;
      if (s == 0.0) continue;
      for (int i = 0; i < m; ++i) qj[i] -= s * v[i];
    }
  }
  // 3. implicit symmetric QR with Wilkinson shift on (d, e)
  const double eps = 2.220446049250313e-16;
  int hi = n - 1;
  int guard = 0;
  const int max_steps = 60 * n;
  while (hi > 0) {
    if (std::fabs(e[hi - 1]) <= eps * (std::fabs(d[hi - 1]) + std::fabs(d[hi]))) {
      e[hi - 1] = 0.0;
      --hi;
      continue;
    }
    int lo = hi - 1;
    while (lo > 0 &&
           std::fabs(e[lo - 1]) > eps * (std::fabs(d[lo - 1]) + std::fabs(d[lo])))
      --lo;
    if (++guard > max_steps) return false;
    const double dd = 0.5 * (d[hi - 1] - d[hi]);
    const double eh = e[hi - 1];
    const double den = dd + ((dd >= 0.0) ? 1.0 : -1.0) * std::hypot(dd, eh);
    const double mu = d[hi] - eh * eh / den;
    double x = d[lo] - mu, z = e[lo];
    for (int k = lo; k < hi; ++k) {
      const double r = std::hypot(x, z);
      double c = 1.0, s = 0.0;
      if (r != 0.0) {
        c = x / r;
        s = -z / r;
      }
      if (k > lo) e[k - 1] = c * x - s * z;
      const double ak = d[k], bk = d[k + 1], fk = e[k];
      d[k] = c * c * ak - 2.0 * c * s * fk + s * s * bk;
      d[k + 1] = s * s * ak + 2.0 * c * s * fk + c * c * bk;
      e[k] = c * s * (ak - bk) + (c * c - s * s) * fk;
      if (k + 1 < hi) {
        const double h = e[k + 1];
        z = -s * h;
        e[k + 1] = c * h;
        x = e[k];
      }
      double* qk = Q.data() + (size_t)k * n;
      double* qk1 = Q.data() + (size_t)(k + 1) * n;
      for (int i = 0; i < n; ++i) {
        const double u = qk[i], t = qk1[i];
        qk[i] = c * u - s * t;
        qk1[i] = s * u + c * t;
      }
    }
  }
  // 4. sort ascending
  std::vector<int> ord(n);
  std::iota(ord.begin(), ord.end(), 0);
  std::stable_sort(ord.begin(), ord.end(), [&](int i, int j) { return d[i] < d[j]; });
  for (int j = 0; j < n; ++j) {
    w[j] = d[ord[j]];
    std::copy(Q.data() + (size_t)ord[j] * n, Q.data() + (size_t)(ord[j] + 1) * n,
              a + (size_t)j * n);
  }
  return true;
}

// Householder QR of the r x c matrix a (column-major).  On return the first
// min(r, c) rows of a hold R (upper trapezoidal; entries below the diagonal
// are zeroed), so that R^T R = A^T A.
inline void qr_r(int r, int c, double* a) {
  const int kmax = std::min(r - 1, c);
  std::vector<double> v(r);
  for (int k = 0; k < kmax; ++k) {
    const int m = r - k;
    double* col = a + (size_t)k * r + k;
    std::copy(col, col + m, v.begin());
    double beta, alpha;
    householder(m, v.data(), beta, alpha);
    if (beta == 0.0) continue;
    col[0] = alpha;
    for (int i = 1; i < m; ++i) col[i] = 0.0;
    for (int j = k + 1; j < c; ++j) {
      double* cj = a + (size_t)j * r + k;
      double s = 0.0;
      for (int i = 0; i < m; ++i) s += v[i] * cj[i];
      s *= beta;
      if (s == 0.0) continue;
      for (int i = 0; i < m; ++i) cj[i] -= s * v[i];
    }
  }
  for (int j = 0; j < c; ++j)
    for (int i = j + 1; i < r; ++i) a[(size_t)j * r + i] = 0.0;
}

// Dot product of two contiguous vectors (fixed summation order: eight
// interleaved partial sums, then the tail), with AVX2 fused multiply-adds.
inline double dotv(int n, const double* a, const double* b) {
  __m256d s0 = _mm256_setzero_pd(), s1 = _mm256_setzero_pd();
  int i = 0;
  for (; i + 8 <= n; i += 8) {
    s0 = _mm256_fmadd_pd(_mm256_loadu_pd(a + i), _mm256_loadu_pd(b + i), s0);
    s1 = _mm256_fmadd_pd(_mm256_loadu_pd(a + i + 4), _mm256_loadu_pd(b + i + 4), s1);
  }
  double t[4];
  _mm256_storeu_pd(t, _mm256_add_pd(s0, s1));
  double s = (t[0] + t[1]) + (t[2] + t[3]);
  for (; i < n; ++i) s += a[i] * b[i];
  return s;
}

// Plane rotation with [c s; -s c] [a; b] = [r; 0].
inline void givens(double a, double b, double& c, double& s, double& r) {
  if (b == 0.0) {
    c = 1.0;
    s = 0.0;
    r = a;
  } else if (a == 0.0) {
    c = 0.0;
    s = 1.0;
    r = b;
  } else {
    r = std::hypot(a, b);
    c = a / r;
    s = b / r;
  }
}

// Singular values of the upper bidiagonal matrix (d, e) of order n by the
// implicit-shift QR iteration of Golub and Kahan (Golub & Van Loan, sec.
// 8.6.2: Wilkinson shift from the trailing 2 x 2 block of B^T B, a bulge
// chased down by alternating right and left rotations, deflation at
// negligible superdiagonal entries, and a zero diagonal entry removed by left
// rotations along its row).  Every left rotation is applied to the rows of W
// (n x nw, row-major), so W ends as U^T W0 with U the left singular vectors.
// On return d holds the singular values with signs.  False if the iteration
// does not converge.
inline bool bidiag_svd(int n, double* d, double* e, double* W, int nw) {
  const double eps = 2.220446049250313e-16;
  double bnorm = 0.0;
  for (int i = 0; i < n; ++i) {
    const double t = std::abs(d[i]) + (i + 1 < n ? std::abs(e[i]) : 0.0);
    if (!std::isfinite(t)) return false;
    bnorm = std::max(bnorm, t);
  }
  if (bnorm == 0.0) return true;
  auto rot_rows = [&](int i, int j, double c, double s) {   // (Wi, Wj) <- G (Wi, Wj)
    double* a = W + (size_t)i * nw;
    double* b = W + (size_t)j * nw;
    for (int t = 0; t < nw; ++t) {
      const double x = a[t], y = b[t];
      a[t] = c * x + s * y;
      b[t] = -s * x + c * y;
    }
  };
  int hi = n - 1;
  long iter = 0;
  const long maxit = 40L * n * n + 1000;
  while (hi > 0) {
    if (++iter > maxit) return false;
    // negligible superdiagonal: relative to its neighbours, or below the
    // rounding level of the whole matrix (the singular values are needed to
    // absolute accuracy eps ||B|| only; a relative test alone converges
    // slowly on the clusters of tiny values of a rank-deficient matrix)
    for (int i = 0; i < hi; ++i)
      if (std::abs(e[i]) <= eps * (std::abs(d[i]) + std::abs(d[i + 1])) ||
          std::abs(e[i]) <= eps * bnorm)
        e[i] = 0.0;
    while (hi > 0 && e[hi - 1] == 0.0) --hi;
    if (hi == 0) break;
    int lo = hi - 1;
    while (lo > 0 && e[lo - 1] != 0.0) --lo;
    // a negligible diagonal entry: zero its row's superdiagonal from the left
    int zi = -1;
    for (int i = lo; i < hi; ++i)
      if (std::abs(d[i]) <= eps * bnorm) {
        zi = i;
        break;
      }
    if (zi >= 0) {
      d[zi] = 0.0;
      double x = e[zi];
      e[zi] = 0.0;
      for (int j = zi + 1; j <= hi && x != 0.0; ++j) {
        double c, s, r;
        givens(d[j], x, c, s, r);
        d[j] = r;
        rot_rows(j, zi, c, s);
        if (j < hi) {
          x = -s * e[j];
          e[j] = c * e[j];
        }
      }
      continue;
    }
    // Golub-Kahan step on rows/columns lo..hi
    const double dm = d[hi - 1], dn = d[hi], em = e[hi - 1], el = hi - 1 > lo ? e[hi - 2] : 0.0;
    const double t11 = dm * dm + el * el, t12 = dm * em, t22 = dn * dn + em * em;
    const double dd = 0.5 * (t11 - t22);
    double mu;
    if (t12 == 0.0)
      mu = t22;
    else
      mu = t22 - t12 * t12 / (dd + (dd >= 0.0 ? 1.0 : -1.0) * std::hypot(dd, t12));
    double y = d[lo] * d[lo] - mu, z = d[lo] * e[lo];
    for (int k = lo; k < hi; ++k) {
      double c, s, r;
      givens(y, z, c, s, r);                 // right rotation of columns k, k+1
      if (k > lo) e[k - 1] = r;
      const double dk = c * d[k] + s * e[k];
      const double ek = -s * d[k] + c * e[k];
      const double bulge = s * d[k + 1];
      d[k + 1] *= c;
      d[k] = dk;
      e[k] = ek;
      givens(d[k], bulge, c, s, r);          // left rotation of rows k, k+1
      d[k] = r;
      const double ek2 = c * e[k] + s * d[k + 1];
      const double dk1 = -s * e[k] + c * d[k + 1];
      e[k] = ek2;
      d[k + 1] = dk1;
      rot_rows(k, k + 1, c, s);
      if (k + 1 < hi) {
        z = s * e[k + 1];
        e[k + 1] *= c;
        y = e[k];
      }
    }
  }
  return true;
}

// The same Schur complement with the range of Bg truncated by its SVD
// (singular values at or below rtol times the largest count as null), which
// does not depend on the basis of Bg's columns.  B (rows x (nw + ng),
// column-major, leading dimension rows, Bw first) is overwritten; S is
// nw x nw, column-major.  Returns the rank kept, or -1 if the SVD iteration
// did not converge.
//
// Only orthogonal transformations are used, so ||B u|| and the singular
// values of Bg are those of the input: rows beyond nw + ng are folded into
// the R factor of B's QR; with fewer rows than Gamma columns, Bg is replaced
// by the triangle L of Bg = [L 0] Q (right transformations leave the left
// singular vectors alone); Householder bidiagonalisation X = U_B [D; 0] V_B^T
// (Golub & Van Loan, sec. 5.4.8) and the Golub-Kahan iteration then give
// the singular values, with every left transformation applied to Bw as well.
// Bw then holds U^T Bw: row j is u_j^T Bw, so S = sum over the dropped
// singular directions (and the rows outside range(Bg)) of its rows' outer
// products -- E^T E with E = (I - U_r U_r^T) Bw -- and U itself is never
// formed.
inline int schur_svd(int rows, int nw, int ng, double* B, double rtol, double* S) {
  const int c = nw + ng;
  int m = rows;
  std::vector<double> R;
  const double* M = B;
  if (rows > c) {
    qr_r(rows, c, B);
    R.resize((size_t)c * c);
    for (int j = 0; j < c; ++j)
      std::copy(B + (size_t)j * rows, B + (size_t)j * rows + c, R.begin() + (size_t)j * c);
    M = R.data();
    m = c;
  }
  std::vector<double> E(M, M + (size_t)nw * m);            // Bw (column-major, m x nw)
  std::vector<char> keep(m, 0);
  int r = 0;
  if (ng > 0) {
    int n = ng;
    std::vector<double> X;
    if (m >= ng) {
      X.assign(M + (size_t)nw * m, M + (size_t)c * m);       // m x n
    } else {                                                // Bg^T = Q' R'  ->  L = R'^T
      std::vector<double> Xt((size_t)ng * m);
      for (int j = 0; j < ng; ++j)
        for (int i2 = 0; i2 < m; ++i2) Xt[(size_t)i2 * ng + j] = M[(size_t)(nw + j) * m + i2];
      qr_r(ng, m, Xt.data());
      n = m;
      X.assign((size_t)m * m, 0.0);
      for (int j = 0; j < m; ++j)
        for (int i2 = j; i2 < m; ++i2) X[(size_t)j * m + i2] = Xt[(size_t)i2 * ng + j];
    }
    std::vector<double> d(n), e(std::max(n - 1, 1), 0.0), v(std::max(m, n)), w(m);
    for (int j = 0; j < n; ++j) {
      {                                                     // left reflector, column j
        const int mm = m - j;
        double* col = X.data() + (size_t)j * m + j;
        std::copy(col, col + mm, v.begin());
        double beta, alpha;
        householder(mm, v.data(), beta, alpha);
        if (beta != 0.0) {
          col[0] = alpha;
          for (int i2 = 1; i2 < mm; ++i2) col[i2] = 0.0;
          auto reflect = [&](double* cj) {
            const double sd = beta * dotv(mm, v.data(), cj);
            if (sd == 0.0) return;
            for (int i2 = 0; i2 < mm; ++i2) cj[i2] -= sd * v[i2];
          };
          for (int q = j + 1; q < n; ++q) reflect(X.data() + (size_t)q * m + j);
          for (int q = 0; q < nw; ++q) reflect(E.data() + (size_t)q * m + j);
        }
        d[j] = X[(size_t)j * m + j];
      }
      if (j + 1 < n) {                                      // right reflector, row j
        const int len = n - j - 1;
        for (int q = 0; q < len; ++q) v[q] = X[(size_t)(j + 1 + q) * m + j];
        double beta, alpha;
        householder(len, v.data(), beta, alpha);
        if (beta != 0.0) {
          // rows j+1.. of the trailing columns: Xs <- Xs (I - beta v v^T)
          const int mr = m - j - 1;
          std::fill(w.begin(), w.begin() + mr, 0.0);
          for (int q = 0; q < len; ++q) {
            const double vq = v[q];
            if (vq == 0.0) continue;
            const double* xq = X.data() + (size_t)(j + 1 + q) * m + j + 1;
            for (int i2 = 0; i2 < mr; ++i2) w[i2] += vq * xq[i2];
          }
          for (int q = 0; q < len; ++q) {
            const double f = beta * v[q];
            if (f == 0.0) continue;
            double* xq = X.data() + (size_t)(j + 1 + q) * m + j + 1;
            for (int i2 = 0; i2 < mr; ++i2) xq[i2] -= f * w[i2];
          }
          X[(size_t)(j + 1) * m + j] = alpha;
          for (int q = 1; q < len; ++q) X[(size_t)(j + 1 + q) * m + j] = 0.0;
        }
        e[j] = X[(size_t)(j + 1) * m + j];
      }
    }
    // rows of U_B^T Bw (row-major) for the QR iteration's left rotations
    std::vector<double> Wr((size_t)n * nw);
    for (int q = 0; q < nw; ++q)
      for (int i2 = 0; i2 < n; ++i2) Wr[(size_t)i2 * nw + q] = E[(size_t)q * m + i2];
    if (!bidiag_svd(n, d.data(), e.data(), Wr.data(), nw)) return -1;
    double smax = 0.0;
    for (int j = 0; j < n; ++j) smax = std::max(smax, std::abs(d[j]));
    for (int j = 0; j < n; ++j) {
      const double sj = std::abs(d[j]);
      if (sj > rtol * smax && sj != 0.0) {
        keep[j] = 1;
        ++r;
      }
      for (int q = 0; q < nw; ++q) E[(size_t)q * m + j] = Wr[(size_t)j * nw + q];
    }
  }
  // S = sum over the rows of U^T Bw that are not kept
  std::vector<double> Ed;
  Ed.reserve((size_t)(m - r) * nw);
  int md = 0;
  for (int i2 = 0; i2 < m; ++i2) md += !keep[i2];
  Ed.assign((size_t)md * nw, 0.0);
  for (int q = 0; q < nw; ++q) {
    int t = 0;
    for (int i2 = 0; i2 < m; ++i2)
      if (!keep[i2]) Ed[(size_t)q * md + t++] = E[(size_t)q * m + i2];
  }
  for (int j = 0; j < nw; ++j) {
    const double* cj = Ed.data() + (size_t)j * md;
    for (int i = j; i < nw; ++i) {
      const double sd = dotv(md, Ed.data() + (size_t)i * md, cj);
      S[(size_t)j * nw + i] = sd;
      S[(size_t)i * nw + j] = sd;
    }
  }
  return r;
}

}  // namespace lsamg

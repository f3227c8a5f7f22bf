// Host real Schur decomposition A = Z T Z^T (FP64), used by the Schur-basis
// seed solve when the eigenbasis is ill-conditioned.
//
// Method: Householder reduction to upper Hessenberg form, then the implicit
// double-shift (Francis) QR iteration with deflation on the active window and
// exceptional shifts, with all transformations accumulated into Z (Golub and
// Van Loan, Matrix Computations, sections 7.4-7.5).  2x2 diagonal blocks with
// real eigenvalues are split by a rotation, so every remaining 2x2 block holds
// a complex-conjugate pair (standard real Schur form).
#include "schur_host.h"

#include <algorithm>
#include <cmath>
#include <vector>

namespace lyap {

namespace {

struct Mat {
  int n;
  std::vector<double> a;  // column-major
  explicit Mat(int n_) : n(n_), a((size_t)n_ * n_, 0.0) {}
  double& operator()(int i, int j) { return a[(size_t)j * n + i]; }
  double operator()(int i, int j) const { return a[(size_t)j * n + i]; }
};

// Apply the reflector P = I - tau v v^T (v of length len, acting on rows/cols
// r0 .. r0+len-1) from the left to H[:, c0:c1] and from the right to H[r0:r1, :]
void refl_left(Mat& H, const double* v, int len, double tau, int r0, int c0, int c1) {
  for (int j = c0; j < c1; ++j) {
    double s = 0;
    for (int k = 0; k < len; ++k) s += v[k] * H(r0 + k, j);
    s *= tau;
    for (int k = 0; k < len; ++k) H(r0 + k, j) -= s * v[k];
  }
}
void refl_right(Mat& H, const double* v, int len, double tau, int c0, int r0, int r1) {
  for (int i = r0; i < r1; ++i) {
    double s = 0;
    for (int k = 0; k < len; ++k) s += H(i, c0 + k) * v[k];
    s *= tau;
    for (int k = 0; k < len; ++k) H(i, c0 + k) -= s * v[k];
  }
}

// Householder vector for x (length len): returns tau, v with v[0] = 1,
// such that (I - tau v v^T) x = beta e1.
double house(const double* x, int len, double* v, double& beta) {
  double sigma = 0;
  for (int k = 1; k < len; ++k) sigma += x[k] * x[k];
  v[0] = 1.0;
  for (int k = 1; k < len; ++k) v[k] = x[k];
  if (sigma == 0.0) {
    beta = x[0];
    return 0.0;
  }
  const double mu = std::sqrt(x[0] * x[0] + sigma);
  const double v0 = x[0] <= 0 ? x[0] - mu : -sigma / (x[0] + mu);
  const double tau = 2 * v0 * v0 / (sigma + v0 * v0);
  for (int k = 1; k < len; ++k) v[k] /= v0;
  beta = mu;
  return tau;
}

void rot_rows(Mat& H, int i, int k, double c, double s, int c0, int c1) {
  for (int j = c0; j < c1; ++j) {
    const double a = H(i, j), b = H(k, j);
    H(i, j) = c * a + s * b;
    H(k, j) = -s * a + c * b;
  }
}
void rot_cols(Mat& H, int i, int k, double c, double s, int r0, int r1) {
  for (int r = r0; r < r1; ++r) {
    const double a = H(r, i), b = H(r, k);
    H(r, i) = c * a + s * b;
    H(r, k) = -s * a + c * b;
  }
}

// Split a 2x2 block at (k, k+1) with real eigenvalues into upper-triangular form.
void standardize(Mat& H, Mat& Z, int k) {
  const int n = H.n;
  const double a = H(k, k), b = H(k, k + 1), c = H(k + 1, k), d = H(k + 1, k + 1);
  if (c == 0.0) return;
  const double p = 0.5 * (a - d);
  const double disc = p * p + b * c;
  if (disc < 0) return;  // complex pair: keep the 2x2 block
  // eigenvalue lambda = d + p +- sqrt(disc); eigenvector (lambda - d, c)
  const double sq = std::sqrt(disc);
  const double lam = (p >= 0) ? d + p + sq : d + p - sq;
  double x = lam - d, y = c;
  // rotation G with G^T [x; y] ~ e1: columns (x, y)/||.|| is the eigenvector
  const double nr = std::hypot(x, y);
  if (nr == 0.0) return;
  const double cs = x / nr, sn = y / nr;
  rot_rows(H, k, k + 1, cs, sn, 0, n);
  rot_cols(H, k, k + 1, cs, sn, 0, n);
  rot_cols(Z, k, k + 1, cs, sn, 0, n);
  H(k + 1, k) = 0.0;
}

}  // namespace

bool real_schur(int n, const double* A_rowmajor, double* T_rowmajor, double* Z_rowmajor,
                int* iterations) {
  Mat H(n), Z(n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) H(i, j) = A_rowmajor[(size_t)i * n + j];
  for (int i = 0; i < n; ++i) Z(i, i) = 1.0;
  std::vector<double> v(n), x(n);

  // ---- Hessenberg reduction ----
  for (int k = 0; k + 2 < n; ++k) {
    const int len = n - k - 1;
    for (int i = 0; i < len; ++i) x[i] = H(k + 1 + i, k);
    double beta;
    const double tau = house(x.data(), len, v.data(), beta);
    if (tau == 0.0) continue;
    refl_left(H, v.data(), len, tau, k + 1, k, n);
    refl_right(H, v.data(), len, tau, k + 1, 0, n);
    refl_right(Z, v.data(), len, tau, k + 1, 0, n);
    for (int i = k + 2; i < n; ++i) H(i, k) = 0.0;
  }

  // ---- Francis double-shift QR ----
  const double eps = 2.220446049250313e-16;
  int hi = n - 1;
  int iter = 0, total = 0;
  const int max_total = 100 * std::max(n, 10);
  while (hi >= 0) {
    if (total > max_total) return false;
    // find the start lo of the unreduced block ending at hi
    int lo = hi;
    while (lo > 0) {
      const double s = std::fabs(H(lo - 1, lo - 1)) + std::fabs(H(lo, lo));
      if (std::fabs(H(lo, lo - 1)) <= eps * (s == 0.0 ? 1.0 : s)) {
        H(lo, lo - 1) = 0.0;
        break;
      }
      --lo;
    }
    if (lo == hi) {  // 1x1 deflation
      --hi;
      iter = 0;
      continue;
    }
    if (lo == hi - 1) {  // 2x2 deflation
      standardize(H, Z, hi - 1);
      hi -= 2;
      iter = 0;
      continue;
    }
    ++iter;
    ++total;
    // shifts: eigenvalues of the trailing 2x2 (as sum and product)
    double s, t;
    if (iter % 11 == 10) {  // exceptional shift
      const double w = std::fabs(H(hi, hi - 1)) + std::fabs(H(hi - 1, hi - 2));
      s = 1.5 * w + H(hi, hi);
      t = w * w;
    } else {
      const double a = H(hi - 1, hi - 1), b = H(hi - 1, hi), c = H(hi, hi - 1), d = H(hi, hi);
      s = a + d;
      t = a * d - b * c;
    }
    // first column of (H - s1 I)(H - s2 I)
    double x0 = H(lo, lo) * H(lo, lo) + H(lo, lo + 1) * H(lo + 1, lo) - s * H(lo, lo) + t;
    double y0 = H(lo + 1, lo) * (H(lo, lo) + H(lo + 1, lo + 1) - s);
    double z0 = H(lo + 1, lo) * H(lo + 2, lo + 1);
    for (int k = lo; k <= hi - 2; ++k) {
      double xv[3] = {x0, y0, z0}, vv[3], beta;
      const double tau = house(xv, 3, vv, beta);
      const int cstart = std::max(lo, k - 1);
      if (tau != 0.0) {
        refl_left(H, vv, 3, tau, k, cstart, n);
        const int rend = std::min(k + 4, hi + 1);
        refl_right(H, vv, 3, tau, k, 0, rend);
        refl_right(Z, vv, 3, tau, k, 0, n);
      }
      x0 = H(k + 1, k);
      y0 = H(k + 2, k);
      if (k < hi - 2) z0 = H(k + 3, k);
    }
    {
      // final 2-element reflector
      double xv[2] = {x0, y0}, vv[2], beta;
      const int k = hi - 1;
      const double tau = house(xv, 2, vv, beta);
      if (tau != 0.0) {
        refl_left(H, vv, 2, tau, k, std::max(lo, k - 1), n);
        refl_right(H, vv, 2, tau, k, 0, hi + 1);
        refl_right(Z, vv, 2, tau, k, 0, n);
      }
    }
    // clean the sub-sub-diagonal of the active window
    for (int i = lo + 2; i <= hi; ++i)
      for (int j = lo; j < i - 1; ++j) H(i, j) = 0.0;
  }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      T_rowmajor[(size_t)i * n + j] = (i > j + 1) ? 0.0 : H(i, j);
      Z_rowmajor[(size_t)i * n + j] = Z(i, j);
    }
  if (iterations) *iterations = total;
  return true;
}

}  // namespace lyap

// Host-side solver set-up: the App. C coefficient fit, the Courant limit from
// the operator symbols, and the FIR taps of the J1 correction.
#include "solver_setup.h"

#include <cmath>
#include <vector>

namespace relpic {

static const double kPi = 3.14159265358979323846;

// Dense Gaussian elimination with partial pivoting; returns false if singular.
static bool solve_dense(std::vector<double> A, std::vector<double> b, int n, std::vector<double> &x) {
  for (int k = 0; k < n; ++k) {
    int piv = k;
    for (int i = k + 1; i < n; ++i)
      if (std::fabs(A[i * n + k]) > std::fabs(A[piv * n + k])) piv = i;
    if (A[piv * n + k] == 0.0) return false;
    if (piv != k) {
      for (int j = 0; j < n; ++j) std::swap(A[k * n + j], A[piv * n + j]);
      std::swap(b[k], b[piv]);
    }
    for (int i = k + 1; i < n; ++i) {
      const double m = A[i * n + k] / A[k * n + k];
      if (m == 0.0) continue;
      for (int j = k; j < n; ++j) A[i * n + j] -= m * A[k * n + j];
      b[i] -= m * b[k];
    }
  }
  x.assign(n, 0.0);
  for (int i = n - 1; i >= 0; --i) {
    double s = b[i];
    for (int j = i + 1; j < n; ++j) s -= A[i * n + j] * x[j];
    x[i] = s / A[i * n + i];
  }
  return true;
}

// App. C: minimize int_0^{1/2} w(k) (sum_l C_l sin((2l-1) pi k)/pi - T(k))^2 dk
// with T(k) = kappa sin(pi k / kappa)/pi, subject to the order-p consistency
// rows, via the Lagrange (KKT) system.  The integrals use the trapezoid rule
// on `nq` intervals of [0, 1/2].
bool fit_axial_coefficients(double kappa, int M, int p, double wk1, double nsg, int nq, std::vector<double> &C,
                            int target_kind) {
  if (target_kind != 0 && target_kind != 1) return false;
  if (M < 1 || p < 2 || (p % 2) || p / 2 > M || kappa <= 1.0 || nq < 16) return false;
  const int r = p / 2;
  const int n = M + r;
  std::vector<double> A(n * n, 0.0), b(n, 0.0);
  std::vector<double> s(M);
  for (int q = 0; q <= nq; ++q) {
    const double k = 0.5 * q / nq;
    double wq = 0.5 / nq;
    if (q == 0 || q == nq) wq *= 0.5;
    const double w = std::exp(-std::log(2.0) * std::pow(2.0 * k / wk1, nsg)) * wq;
    // 0: [k1]_t; 1: [k1]_t^2 / [k]_Yee (the operator on E when the one on B is Yee)
    double target = kappa * std::sin(kPi * k / kappa) / kPi;
    if (target_kind == 1) target = k == 0.0 ? 0.0 : target * target / (std::sin(kPi * k) / kPi);
    for (int i = 0; i < M; ++i) s[i] = std::sin((2 * i + 1) * kPi * k);
    for (int i = 0; i < M; ++i) {
      b[i] += (2.0 / kPi) * w * s[i] * target;
      for (int j = 0; j < M; ++j) A[i * n + j] += (2.0 / (kPi * kPi)) * w * s[i] * s[j];
    }
  }
  for (int i = 1; i <= r; ++i) {
    double fact = 1.0;
    for (int t = 2; t <= 2 * i - 1; ++t) fact *= t;
    for (int j = 1; j <= M; ++j) {
      const double v = std::pow(2.0 * j - 1.0, 2 * i - 1) / fact;
      A[(M + i - 1) * n + (j - 1)] = v;
      A[(j - 1) * n + (M + i - 1)] = v;
    }
    b[M + i - 1] = (i == 1) ? 1.0 : 0.0;
  }
  std::vector<double> x;
  if (!solve_dense(A, b, n, x)) return false;
  C.assign(x.begin(), x.begin() + M);
  return true;
}

double axial_symbol_max(const double *C, int M) {
  // max over khat in [0, pi/2] of |sum_l C_l sin((2l-1) khat)|
  double best = 0.0;
  const int ns = 8192;
  for (int q = 0; q <= ns; ++q) {
    const double kh = 0.5 * kPi * q / ns;
    double v = 0.0;
    for (int l = 1; l <= M; ++l) v += C[l - 1] * std::sin((2 * l - 1) * kh);
    best = std::fmax(best, std::fabs(v));
  }
  return best;
}

double axial_product_max(const double *CE, const double *CB, int M) {
  // max over khat in [0, pi/2] of |sigma_E(khat) sigma_B(khat)|
  double best = 0.0;
  const int ns = 8192;
  for (int q = 0; q <= ns; ++q) {
    const double kh = 0.5 * kPi * q / ns;
    double a = 0.0, b = 0.0;
    for (int l = 1; l <= M; ++l) {
      a += CE[l - 1] * std::sin((2 * l - 1) * kh);
      b += CB[l - 1] * std::sin((2 * l - 1) * kh);
    }
    best = std::fmax(best, std::fabs(a * b));
  }
  return best;
}

double courant_number(int ndim, const double *dx, double dt, const double *C, int M) {
  return courant_number2(ndim, dx, dt, C, C, M);
}

double courant_number2(int ndim, const double *dx, double dt, const double *CE, const double *CB, int M) {
  double sum = axial_product_max(CE, CB, M) / (dx[0] * dx[0]);
  for (int d = 1; d < ndim; ++d) sum += 1.0 / (dx[d] * dx[d]);
  return dt * std::sqrt(sum);  // (dt/2) * sqrt(sum (2 sigma_d / dx_d)^2)
}

// The customized backward difference telescopes into the Yee one:
// d-_custom = K * d-_Yee with K_m = sum_{l > |m|} C_l, |m| <= M-1.  The J1
// correction is G = K^{-1}.  K is symmetric positive definite (its symbol is
// [k]_custom/[k]_Yee > 0), so G decays exponentially.  The taps are the
// central column of the inverse of the banded Toeplitz matrix of K on a line
// of 2L+1 points (banded LU without pivoting, stable for SPD), which equals
// the infinite-line inverse to round-off once L >> the decay length.
bool correction_taps(const double *C, int M, double tol, int max_taps, std::vector<double> &taps) {
  taps.clear();
  if (M <= 1) return true;
  std::vector<double> K(M, 0.0);
  for (int m = 0; m < M; ++m)
    for (int l = m + 1; l <= M; ++l) K[m] += C[l - 1];
  const int L = 512;
  const int n = 2 * L + 1;
  const int bw = M - 1;
  // band storage: row i, columns i-bw..i+bw at offset (j - i + bw)
  const int W = 2 * bw + 1;
  std::vector<double> Bm((size_t)n * W, 0.0);
  for (int i = 0; i < n; ++i)
    for (int j = i - bw; j <= i + bw; ++j)
      if (j >= 0 && j < n) Bm[(size_t)i * W + (j - i + bw)] = K[std::abs(i - j)];
  std::vector<double> rhs(n, 0.0);
  rhs[L] = 1.0;
  for (int k = 0; k < n; ++k) {
    const double piv = Bm[(size_t)k * W + bw];
    if (!(piv > 0.0)) return false;
    for (int i = k + 1; i <= std::min(n - 1, k + bw); ++i) {
      const double m = Bm[(size_t)i * W + (k - i + bw)] / piv;
      if (m == 0.0) continue;
      for (int j = k; j <= std::min(n - 1, k + bw); ++j) Bm[(size_t)i * W + (j - i + bw)] -= m * Bm[(size_t)k * W + (j - k + bw)];
      rhs[i] -= m * rhs[k];
    }
  }
  std::vector<double> x(n, 0.0);
  for (int i = n - 1; i >= 0; --i) {
    double s = rhs[i];
    for (int j = i + 1; j <= std::min(n - 1, i + bw); ++j) s -= Bm[(size_t)i * W + (j - i + bw)] * x[j];
    x[i] = s / Bm[(size_t)i * W + bw];
  }
  int ng = 0;
  for (int m = 1; m < L; ++m)
    if (std::fabs(x[L + m]) >= tol * std::fabs(x[L])) ng = m;
  if (ng > max_taps) return false;
  taps.assign(x.begin() + L, x.begin() + L + ng + 1);
  return true;
}

}  // namespace relpic
